"""Parity of the HIP path with the FP64 oracle, called through the C ABI.

One-step parity (km_assign, km_step) over a sweep of d and k at ragged n,
adversarial ties and empty clusters, BF16 input, the sampler's index lists,
end-to-end two-stage fits on every workload family at reduced n, determinism,
and the 10M x 16 workload at full size on sampled outputs.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import (CTOL, GAP, JTOL, j_atol, assert_centers, assert_labels, assert_step,
                         exempt_mask, sums_from_labels, to_device, widen)

pytestmark = pytest.mark.gpu

km = pytest.importorskip("paper_1108_1351_amd")


def _mixture(n, d, k, seed, dtype="f32", spread=20.0):
    spec = synth.MixtureSpec(d, k, "uniform", -spread, spread, sigma_lo=0.5, sigma_hi=2.0,
                             weights="dirichlet1")
    return synth.generate(spec, seed, n, dtype)


def _centers_from(Xh, k, seed, jitter=0.3):
    rng = np.random.default_rng(seed)
    rows = rng.choice(len(Xh), size=k, replace=len(Xh) < k)
    return widen(Xh)[rows] + rng.normal(0.0, jitter, size=(k, Xh.shape[1]))


# ------------------------------------------------------------------ sampling
@pytest.mark.parametrize("n,m,k,seed", [(1, 1, 1, 0), (100, 10, 3, 5), (10_007, 101, 8, 7),
                                        (100_000, 1000, 8, 1), (1 << 20, 4096, 64, 11),
                                        (3_000_000, 3000, 1024, 2**64 - 1),
                                        (10_000_000, 100_000, 64, 2), (5000, 5000, 17, 9)])
def test_sample_matches_oracle(n, m, k, seed):
    print(f"[sample] n={n} m={m} k={k}", flush=True)
    sub, ini = km.km_sample(n, m, k, seed)
    rsub, rini = oracle.select(n, m, k, seed)
    assert np.array_equal(sub.cpu().numpy(), rsub)
    assert np.array_equal(ini.cpu().numpy(), rini)


# ------------------------------------------------------------ one-step parity
SWEEP = [(1, 1), (1, 5), (2, 8), (3, 3), (4, 32), (5, 7), (8, 64), (16, 64), (17, 31),
         (16, 1024), (32, 8), (32, 257), (64, 64), (100, 100), (128, 2), (128, 1024),
         (129, 16), (200, 33), (2, 2000), (8, 5000), (300, 40), (1000, 3)]


@pytest.mark.parametrize("d,k", SWEEP)
def test_assign_parity(d, k):
    n = 10_007
    print(f"[assign] n={n} d={d} k={k}", flush=True)
    Xh = _mixture(n, d, min(k, 50), seed=d * 1000 + k)
    C = _centers_from(Xh, k, seed=k)
    lab, J, unc = km.km_assign(to_device(Xh), torch.from_numpy(C).cuda())
    ex = assert_labels(lab, Xh, C, name=f"assign d={d} k={k}")
    rlab, D1, _ = oracle.assign(Xh, C)
    assert abs(J - D1.sum()) <= 1e-12 * D1.sum()
    assert ex <= 2


@pytest.mark.parametrize("d,k", SWEEP)
def test_step_parity(d, k):
    n = 10_007
    print(f"[step] n={n} d={d} k={k}", flush=True)
    Xh = _mixture(n, d, min(k, 50), seed=d * 7 + k)
    C = _centers_from(Xh, k, seed=k + 1)
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda())
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, name=f"step d={d} k={k}")


SMALL_D = [(1, 5), (2, 8), (4, 32), (5, 7), (8, 64), (16, 64), (16, 128), (3, 100)]


@pytest.mark.parametrize("d,k", SMALL_D)
@pytest.mark.parametrize("precision", ["auto", "bf16_rerank", "fp32"])
def test_small_d_fused_paths(d, k, precision):
    """d <= 16, k <= 128: the fused pass on the split BF16 screen (auto), on the
    plain BF16 screen (bf16_rerank) and on FP32 MFMA (fp32) give the oracle's
    labels, J and new centers."""
    n = 20_011
    print(f"[small-d {precision}] n={n} d={d} k={k}", flush=True)
    Xh = _mixture(n, d, min(k, 40), seed=d * 31 + k)
    C = _centers_from(Xh, k, seed=k + 5, jitter=0.5)
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda(), precision=precision)
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, name=f"small-d {precision} d={d} k={k}")
    lab2, J2, _ = km.km_assign(to_device(Xh), torch.from_numpy(C).cuda(), precision=precision)
    assert_step({"labels": lab2, "J": J2}, Xh, C, ref, name="assign")


@pytest.mark.parametrize("d,k,dtype", [(8, 70, "f32"), (12, 90, "f32"), (16, 96, "bf16"),
                                         (4, 33, "bf16"), (7, 128, "bf16"), (2, 3, "f32")])
def test_split_screen_paths(d, k, dtype):
    """The split screen (auto precision, d <= 16, k <= 128) over the shapes its
    kernel is specialised for: 4, 8 or 16 padded dims, one to four 32-center
    tiles, whole or padded rows, FP32 and BF16 data, a ragged last 64-point
    block.  Labels, counts, exact sums (through the new centers) and J as the
    oracle's."""
    n = 30_001
    print(f"[split paths] n={n} d={d} k={k} {dtype}", flush=True)
    Xh = _mixture(n, d, min(k, 40), seed=d * 7 + k, dtype=dtype)
    C = _centers_from(Xh, k, seed=k + 11, jitter=0.5)
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda())
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, name=f"split d={d} k={k} {dtype}")


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 130])
@pytest.mark.parametrize("k,d", [(1, 4), (2, 1), (3, 16), (5, 9)])
def test_split_screen_tiny_inputs(n, k, d):
    """Degenerate and ragged sizes on the split screen (auto precision): fewer
    points than one 64-point block, one center (always certain), two centers
    (no third key), d = 1 and 9 padded to 4 and 16 dims."""
    if k > n:
        pytest.skip("k > n is rejected")
    rng = np.random.default_rng(n * 13 + k * 7 + d)
    Xh = rng.normal(0, 3.0, size=(n, d)).astype(np.float32)
    C = Xh[rng.choice(n, size=k, replace=False)].astype(np.float64) + 0.25
    print(f"[split tiny] n={n} k={k} d={d}", flush=True)
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda())
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, name=f"split tiny n={n} k={k} d={d}")


@pytest.mark.parametrize("d,k", [(16, 64), (4, 32), (8, 20)])
def test_split_screen_misaligned_rows(d, k):
    """X starting 4 bytes past a 16-byte boundary: the split screen cannot load
    whole rows as aligned vectors and takes its element-load path."""
    n = 10_007
    Xh = _mixture(n, d, min(k, 20), seed=d + k)
    flat = torch.empty(n * d + 1, dtype=torch.float32, device="cuda")
    flat[1:] = torch.from_numpy(Xh.reshape(-1)).cuda()
    X = flat[1:].view(n, d)
    assert X.data_ptr() % 16 == 4
    C = _centers_from(Xh, k, seed=k, jitter=0.5)
    print(f"[split misaligned] n={n} d={d} k={k}", flush=True)
    out = km.km_step(X, torch.from_numpy(C).cuda())
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, name="misaligned")


def test_step_bf16_input():
    Xh = _mixture(20_011, 64, 40, seed=3, dtype="bf16")
    C = _centers_from(Xh, 40, seed=4)
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda())
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, name="bf16 input")


# ---------------------------------------------------------------- adversarial
def test_ties_go_to_lowest_index_and_empties_keep_center():
    # points on the bisector of two centers, duplicated centers, a far center
    xs = np.array([[0.0, y] for y in np.linspace(-3, 3, 301)], np.float32)
    C = np.array([[1.0, 0.0], [-1.0, 0.0], [1.0, 0.0], [1e4, 1e4]])
    out = km.km_step(to_device(xs), torch.from_numpy(C).cuda())
    lab = out["labels"].cpu().numpy()
    assert (lab == 0).all()
    assert out["empty"] == 3 and out["N"].cpu().numpy().tolist() == [301, 0, 0, 0]
    Cn = out["C_new"].cpu().numpy()
    assert np.array_equal(Cn[1:], C[1:])
    assert out["uncertain"] == 301
    ref = oracle.step(xs, C)
    assert np.array_equal(ref.labels, lab) and np.allclose(Cn, ref.C_new, atol=1e-12)


def test_integer_grid_exact_ties():
    g = np.stack(np.meshgrid(np.arange(-8, 9), np.arange(-8, 9)), -1).reshape(-1, 2)
    Xh = np.repeat(g, 3, axis=0).astype(np.float32)
    C = np.array([[-4.0, -4.0], [4.0, -4.0], [-4.0, 4.0], [4.0, 4.0], [0.0, 0.0]])
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda())
    ref = oracle.step(Xh, C)
    assert np.array_equal(out["labels"].cpu().numpy(), ref.labels)
    assert np.array_equal(out["N"].cpu().numpy(), ref.N)
    assert np.allclose(out["C_new"].cpu().numpy(), ref.C_new, rtol=0, atol=1e-12)


def test_nonfinite_input_rejected():
    Xh = _mixture(1000, 4, 3, seed=1)
    Xh[17, 2] = np.nan
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_fit(to_device(Xh), 3, 0.5, 0, 10, 1e-4)
    assert e.value.status == km.KM_EINVAL


# ------------------------------------------------------------------ end to end
# Reduced sizes of the workloads (the full sizes are in test_gpu_fullsize.py).
# The 128-D workload keeps m = 0.005 n = 2048 > k = 1024 subset points, so its
# fast stage clusters a real subset on the BF16 screen (at m = k every subset
# point would be its own center).
FITS = [
    ("gmm2d_n1e5_k8", None),
    ("gmm16d_n1e7_k64", 200_003),
    ("gmm4d_n5e8_k32", 300_007),
    ("gmm128d_n1e8_k1024_bf16", 409_613),
]


def _fit_both(w, Xh, **kw):
    X = to_device(Xh)
    C, L, info = km.kmeans_fit_ex(X, w.k, w.subset_frac, w.fit_seed, w.max_iter, w.tol,
                                  centers64=True, history=True, **kw)
    ref = oracle.fit(Xh, w.k, w.subset_frac, w.fit_seed, w.max_iter, w.tol, **kw)
    return C, L, info, ref


@pytest.mark.parametrize("name,n", FITS)
def test_fit_parity(name, n):
    w = synth.WORKLOADS[name]
    if n is not None:
        w = w.scaled(n)
    print(f"[fit] {w.name} n={w.n} d={w.d} k={w.k}", flush=True)
    Xh = w.data()
    C, L, info, ref = _fit_both(w, Xh)
    C64 = info["centers64"].cpu().numpy()
    assert info["m"] == ref.info["m"]
    assert info["iters"] == ref.info["iters"], (info["iters"], ref.info["iters"])
    assert info["converged"] == ref.info["converged"]
    assert info["empty"] == ref.info["empty"]
    assert info["dist_evals"] == ref.info["dist_evals"]
    assert_centers(C64, ref.centers, Xh, name=w.name)
    assert np.allclose(C.cpu().numpy(), C64.astype(np.float32), rtol=0, atol=0)
    atol = j_atol(Xh)
    assert abs(info["J"] - ref.info["J"]) <= JTOL * ref.info["J"] + atol
    for s in range(2):
        assert np.allclose(info["J_hist"][s], ref.J_hist[s], rtol=JTOL, atol=atol)
    assert abs(info["J_stage1"] - ref.info["J_stage1"]) <= \
        JTOL * ref.info["J_stage1"] + j_atol(Xh)
    assert_labels(L, Xh, ref.centers, ref_labels=ref.labels, name=w.name)
    assert_labels(L, Xh, C64, name=w.name + " at own centers")
    if w.name.startswith("gmm128d"):
        assert ref.info["m"] > w.k  # the fast stage is not degenerate


def test_fit_normal_mode_and_resume():
    w = synth.WORKLOADS["gmm16d_n1e7_k64"].scaled(50_000)
    Xh = w.data()
    C, L, info, ref = _fit_both(w, Xh, skip_stage1=True)
    assert info["iters"][0] == 0 and info["iters"] == ref.info["iters"]
    assert_centers(info["centers64"].cpu().numpy(), ref.centers, Xh)
    # resume the slow stage from given centers (a saved fast-stage result)
    C0 = _centers_from(Xh, w.k, seed=5)
    C, L, info, ref = _fit_both(w, Xh, skip_stage1=True, init_centers=C0)
    assert info["iters"] == ref.info["iters"]
    assert_centers(info["centers64"].cpu().numpy(), ref.centers, Xh)


def test_speedup_sweep_cells_match_oracle():
    """The two-stage vs normal k-means sweep: both fits of a cell run the
    oracle's passes and evaluations, so the evals ratio is the oracle's."""
    import bench
    rows = bench.speedup_sweep(reps=1, max_iter=200, table2_n=20_000, fracs=[0.1],
                               tols=[1e-2, 1e-4], sizes=[30_000], sec61_frac=0.05)
    assert len(rows) == 3
    specs = bench.speedup_specs()
    for row in rows:
        key = "table2" if row["grid"].startswith("table2") else "sec61"
        _, spec, k, seed = specs[key]
        print(f"[speedup] {row['grid']} n={row['n']} tol={row['tol']}", flush=True)
        Xh = synth.generate(spec, seed, row["n"], "f32")
        for mode, normal in (("two_stage", False), ("normal", True)):
            ref = oracle.fit(Xh, k, row["subset_frac"], bench.SPEEDUP_FIT_SEED, row["max_iter"],
                             row["tol"], skip_stage1=normal)
            assert row[mode]["evals"] == ref.info["dist_evals"], (mode, row[mode], ref.info)
            assert abs(row[mode]["J"] - ref.info["J"]) <= JTOL * ref.info["J"] + j_atol(Xh)
        assert row["speedup_evals"] == row["normal"]["evals"] / row["two_stage"]["evals"]


def test_fit_per_stage_tolerances():
    w = synth.WORKLOADS["gmm2d_n1e5_k8"].scaled(30_000)
    Xh = w.data()
    X = to_device(Xh)
    C, L, info = km.kmeans_fit_ex(X, w.k, 0.1, 3, (40, 60), (1e-3, 1e-6), centers64=True)
    ref = oracle.fit(Xh, w.k, 0.1, 3, (40, 60), (1e-3, 1e-6))
    assert info["iters"] == ref.info["iters"]
    assert_centers(info["centers64"].cpu().numpy(), ref.centers, Xh)


def test_deterministic_bits():
    w = synth.WORKLOADS["gmm16d_n1e7_k64"].scaled(100_000)
    X = to_device(w.data())
    a = km.kmeans_fit_ex(X, w.k, w.subset_frac, w.fit_seed, w.max_iter, w.tol, centers64=True)
    b = km.kmeans_fit_ex(X, w.k, w.subset_frac, w.fit_seed, w.max_iter, w.tol, centers64=True)
    assert torch.equal(a[2]["centers64"], b[2]["centers64"])
    assert torch.equal(a[1], b[1])
    assert a[2]["J"] == b[2]["J"] and a[2]["iters"] == b[2]["iters"]


def test_kmeans_fit_plain_entry_point():
    w = synth.WORKLOADS["gmm2d_n1e5_k8"]
    Xh = w.data()
    C, L, info = km.kmeans_fit(to_device(Xh), w.k, w.subset_frac, w.fit_seed, w.max_iter,
                               w.tol)
    ref = oracle.fit(Xh, w.k, w.subset_frac, w.fit_seed, w.max_iter, w.tol)
    assert info["iters"] == ref.info["iters"]
    assert_centers(C.cpu().numpy().astype(np.float64), ref.centers, Xh)
    assert abs(info["J"] - ref.info["J"]) <= JTOL * ref.info["J"]


# ------------------------------------------------------- full-size workload
def test_full_size_16d_sampled_outputs():
    """10M x 16, k = 64, as timed by the benchmark: the oracle checks labels on a
    sample of rows, J over all rows, and one pass at the returned centers."""
    w = synth.WORKLOADS["gmm16d_n1e7_k64"]
    print(f"[full] {w.name}: generating {w.n} x {w.d}", flush=True)
    Xh = w.data()
    X = to_device(Xh)
    C, L, info = km.kmeans_fit_ex(X, w.k, w.subset_frac, w.fit_seed, w.max_iter, w.tol,
                                  centers64=True)
    print(f"[full] fit done iters={info['iters']} uncertain={info['uncertain']}", flush=True)
    C64 = info["centers64"].cpu().numpy()
    lab = L.cpu().numpy()
    rows = np.random.default_rng(0).choice(w.n, 200_000, replace=False)
    rows.sort()
    assert_labels(lab[rows], np.ascontiguousarray(Xh[rows]), C64, name="sampled rows")
    _, D1, _ = oracle.assign(Xh, C64)
    assert abs(info["J"] - D1.sum()) <= JTOL * D1.sum()
    # one pass at the returned centers: identical sums and movement on all rows
    out = km.km_step(X, info["centers64"])
    ref = oracle.step(Xh, C64)
    ex = exempt_mask(Xh[rows], C64)
    assert np.array_equal(out["labels"].cpu().numpy()[rows][~ex], ref.labels[rows][~ex])
    assert_centers(out["C_new"].cpu().numpy(), ref.C_new, Xh, tol=1e-9)
    assert abs(out["J"] - ref.J) <= 1e-12 * ref.J
    if info["converged"][1]:
        assert ref.shift < w.tol * 1.01


@pytest.mark.parametrize("d,k", [(16, 64), (4, 32), (2, 8), (32, 100)])
def test_near_duplicate_centers_resolved_in_fp64(d, k):
    """Pairs of centers closer than the FP32 score quantum (but far above the
    1e-6 near-tie exemption): the FP64 decision must match the oracle on every
    point, including candidates held by the same lane half."""
    rng = np.random.default_rng(d * 31 + k)
    base = rng.uniform(-40, 40, size=(k // 2, d))
    off = rng.normal(size=(k // 2, d))
    off *= 2e-3 / np.linalg.norm(off, axis=1, keepdims=True)
    C = np.empty((k, d))
    C[0::2][:len(base)] = base
    C[1::2][:len(base)] = base + off
    if k % 2:
        C[-1] = rng.uniform(-40, 40, size=d)
    comp = rng.integers(0, k, size=40_000)
    Xh = (C[comp] + rng.normal(0, 1.0, size=(40_000, d))).astype(np.float32)
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda())
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, name=f"near duplicates d={d} k={k}")


# ------------------------------------------------------------- BF16 screen
@pytest.mark.parametrize("d,k,dtype", [(32, 64, "bf16"), (128, 1024, "bf16"), (100, 37, "bf16"),
                                       (64, 300, "f32"), (256, 50, "bf16"), (16, 64, "f32"),
                                       (200, 129, "f32"), (16, 300, "f32"), (8, 200, "bf16")])
def test_bf16_screen_step_parity(d, k, dtype):
    """BF16 MFMA screen, certified candidates, FP32 re-rank and FP64 decisions."""
    n = 12_289
    print(f"[bf16 step] n={n} d={d} k={k} {dtype}", flush=True)
    Xh = _mixture(n, d, min(k, 60), seed=d + 3 * k, dtype=dtype)
    C = _centers_from(Xh, k, seed=k + 7, jitter=0.2)
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda(), precision="bf16_rerank")
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, jtol=1e-9, name=f"bf16 step d={d} k={k} {dtype}")
    lab2, J2, _ = km.km_assign(to_device(Xh), torch.from_numpy(C).cuda(), precision="bf16_rerank")
    assert_step({"labels": lab2, "J": J2}, Xh, C, ref, jtol=1e-9, name="bf16 assign")


@pytest.mark.parametrize("copies", [3, 6, 20])
def test_bf16_screen_crowded_centers(copies):
    """Clusters holding several near-identical centers: more than four candidates
    send points to the re-screen queue; more than sixteen overflow its list and
    the point is decided in FP64 over all centers."""
    d, base = 128, 12
    rng = np.random.default_rng(copies)
    mu = rng.normal(0, 5.0, size=(base, d))
    C = np.repeat(mu, copies, axis=0) + rng.normal(0, 0.05, size=(base * copies, d))
    comp = rng.integers(0, base, size=8_000)
    Xh = synth_bf16(mu[comp] + rng.normal(0, 1.0, size=(8_000, d)))
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda())
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, jtol=1e-9, name=f"crowded x{copies}")


def _far_centers(d, count, seed):
    rng = np.random.default_rng(seed)
    return 40.0 + rng.normal(0, 3.0, size=(count, d))


@pytest.mark.parametrize("d", [128, 16])
@pytest.mark.parametrize("extra", [0, 38])
@pytest.mark.parametrize("m", [0, 5, 40, 100])
def test_bf16_screen_band_covers_center_rounding(m, extra, d):
    """Adversarial BF16 rounding of the centers.  x = (1, ..., 1); c1 and c2 are
    constant vectors just below and just above a BF16 rounding midpoint of -2c,
    so every entry of the screen's copy of c1 rounds up by almost half an ulp
    and every entry of c2's rounds down.  c1 is the nearer center, but the
    screen's scores put c2 ahead by nearly 128 * 2^-6 = 2, more than half of
    the worst-case error of two scores: only a band that covers the full
    rounding of both centers sends the point to the re-rank.  d = 16 runs the
    fused small-d screen, d = 128 the split screen."""
    v1, v2 = 1 + (m + 0.49) * 2.0 ** -7, 1 + (m + 0.51) * 2.0 ** -7
    C = np.vstack([np.full((1, d), v1), np.full((1, d), v2), _far_centers(d, extra, m)])
    Xh = synth_bf16(np.ones((64, d)))
    ref = oracle.step(Xh, C)
    assert (ref.labels == 0).all()
    print(f"[bf16 band] d={d} m={m} k={len(C)}", flush=True)
    lab, J, _ = km.km_assign(to_device(Xh), torch.from_numpy(C).cuda(), precision="bf16_rerank")
    assert (lab.cpu().numpy() == 0).all()
    assert abs(J - ref.J) <= 1e-9 * ref.J


@pytest.mark.parametrize("d", [128, 16])
@pytest.mark.parametrize("extra", [0, 38])
def test_bf16_screen_band_covers_fp32_data_rounding(extra, d):
    """FP32 data whose BF16 roundings all point one way: with c1 = -c2 = 0.5
    (exact in BF16), the rounded point prefers c1 by 0.78 while c2 is nearer;
    the band term 4 ||x^ - x|| max||c|| (about 1.0 at d = 128) catches it."""
    x = np.empty(d, np.float32)
    x[0::2] = np.float32(1 + 0.51 * 2.0 ** -7)
    x[1::2] = np.float32(-(1 + 0.49 * 2.0 ** -7))
    x[1] = np.float32(-1.109375)
    Xh = np.tile(x, (64, 1))
    C = np.vstack([np.full((1, d), 0.5), np.full((1, d), -0.5), _far_centers(d, extra, 3)])
    ref = oracle.step(Xh, C)
    assert (ref.labels == 1).all()
    print(f"[bf16 band f32] d={d} k={len(C)}", flush=True)
    lab, J, _ = km.km_assign(to_device(Xh), torch.from_numpy(C).cuda(), precision="bf16_rerank")
    assert (lab.cpu().numpy() == 1).all()
    assert abs(J - ref.J) <= 1e-9 * ref.J


@pytest.mark.parametrize("d", [16, 8, 4])
@pytest.mark.parametrize("extra", [0, 38])
@pytest.mark.parametrize("m", [128, 190, 255])
def test_split_screen_band_covers_low_part_rounding(m, extra, d):
    """Adversarial rounding of the centers' low BF16 parts (auto precision, small
    d: the split screen).  x = (1, ..., 1) in BF16; -2c = -2 - 2t with 2t just
    below (c1) or above (c2) a rounding midpoint of the low part, so the dropped
    remainders e of the two centers are about -0.49 and +0.49 of the low part's
    ulp in every dim: the screen prefers c2 by about d 2^-16 while c1 is
    nearer (by far less)."""
    u = 2.0 ** -15
    t1, t2 = (m + 0.49) * u / 2, (m + 0.51) * u / 2
    C = np.vstack([np.full((1, d), 1 + t1), np.full((1, d), 1 + t2), _far_centers(d, extra, m)])
    Xh = synth_bf16(np.ones((64, d)))
    ref = oracle.step(Xh, C)
    assert (ref.labels == 0).all()
    print(f"[split band c] d={d} m={m} k={len(C)}", flush=True)
    lab, J, _ = km.km_assign(to_device(Xh), torch.from_numpy(C).cuda(), precision="auto")
    assert (lab.cpu().numpy() == 0).all()
    assert abs(J - ref.J) <= 1e-9 * ref.J


@pytest.mark.parametrize("d", [16, 8, 4])
@pytest.mark.parametrize("extra", [0, 38])
def test_split_screen_band_covers_fp32_low_part_rounding(extra, d):
    """FP32 data whose low BF16 parts all round one way (auto precision, small d:
    the split screen).  x_t = s_t (1 + rho_t) with signs s alternating, so
    x^ = s; rho_t sits 2^-6 of an ulp (u = 2^-16) off a rounding midpoint of the
    low part, so every dropped remainder is (1/2 - 2^-6) u against s_t.  With
    c1 = -c2 = 0.5 (exact in BF16) the screen sees sum(x^ + xlo) > 0 (c1 nearer)
    while sum(x) < 0 (c2 nearer)."""
    u = 2.0 ** -16
    half = d // 2
    mp = np.full(half, 150)
    mm = np.full(half, 150)
    mm[: max(1, (31 * d) // 100)] += 1  # sum over s = -1 of m exceeds that over s = +1
    # offsets 0.5 +- 2^-6 of an ulp: dyadic, so every x_t is exact in FP32
    x = np.empty(d, np.float64)
    x[0::2] = 1 + (mp + 0.5 + 2.0 ** -6) * u
    x[1::2] = -(1 + (mm + 0.5 - 2.0 ** -6) * u)
    xs = x.astype(np.float32)
    assert np.array_equal(xs.astype(np.float64), x)
    Xh = np.tile(xs, (64, 1))
    C = np.vstack([np.full((1, d), 0.5), np.full((1, d), -0.5), _far_centers(d, extra, 3)])
    ref = oracle.step(Xh, C)
    assert x.sum() < 0 and (ref.labels == 1).all()
    print(f"[split band f32] d={d} k={len(C)}", flush=True)
    lab, J, _ = km.km_assign(to_device(Xh), torch.from_numpy(C).cuda(), precision="auto")
    assert (lab.cpu().numpy() == 1).all()
    assert abs(J - ref.J) <= 1e-9 * ref.J


def synth_bf16(A):
    """Round an FP64 array to BF16 bit patterns (nearest, ties to even)."""
    f = A.astype(np.float32).view(np.uint32).astype(np.uint64)
    r = (f + 0x7FFF + ((f >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def test_forced_fp32_path_on_bf16_data():
    Xh = _mixture(9_001, 64, 30, seed=11, dtype="bf16")
    C = _centers_from(Xh, 30, seed=12)
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda(), precision="fp32")
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, jtol=1e-9, name="fp32 on bf16")


def test_step_more_labels_than_lds_counters():
    """More than 16384 clusters: the label sort counts with global atomics."""
    n, d, k = 50_000, 3, 17_000
    Xh = _mixture(n, d, 40, seed=17)
    C = _centers_from(Xh, k, seed=18, jitter=0.3)
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda())
    ref = oracle.step(Xh, C)
    assert_step(out, Xh, C, ref, jtol=1e-9, name="17000 labels")


def test_step_label_sort_ranges_per_chunk():
    """k = 4090 labels over 4.5M rows: the label sort's chunks (4,608 rows) are
    longer than the ranges it sorts in LDS (4,096 rows at this k), so each chunk
    takes two ranges, and the last chunk is ragged.  Labels of sampled rows are
    the oracle's; counts, sums, new centers and J are checked against FP64 sums
    over the GPU's own labels (a point written twice or not at all by the
    scatter would change a cluster's sum by far more than the quantum)."""
    n, d, k = 4_500_001, 16, 4090
    Xh = _mixture(n, d, 60, seed=23)
    C = _centers_from(Xh, k, seed=24, jitter=0.3)
    print(f"[label sort ranges] n={n} d={d} k={k}", flush=True)
    out = km.km_step(to_device(Xh), torch.from_numpy(C).cuda())
    lab = out["labels"].cpu().numpy()
    rows = np.sort(np.random.default_rng(25).choice(n, 20_000, replace=False))
    assert_labels(lab[rows], np.ascontiguousarray(Xh[rows]), C, name="sampled rows")
    S_l, A_l, N_l = sums_from_labels(Xh, lab, k)
    assert np.array_equal(out["N"].cpu().numpy(), N_l)
    X = widen(Xh)
    quantum = 2.0 ** (np.floor(np.log2(np.abs(X).max())) - 29)
    S = out["S"].cpu().numpy()
    assert np.all(np.abs(S - S_l) <= N_l[:, None] * quantum + 1e-12 * A_l)
    C_exp = np.where(N_l[:, None] > 0, S_l / np.maximum(N_l, 1)[:, None], C)
    assert_centers(out["C_new"].cpu().numpy(), C_exp, Xh, tol=1e-9, name="C_new")
    J_l = float(((X - C[lab]) ** 2).sum())
    assert abs(out["J"] - J_l) <= 1e-9 * J_l, (out["J"], J_l)
