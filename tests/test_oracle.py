"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
published SplitMix64 outputs, brute-force enumeration of partitions, closed forms
(k = 1, k = n, 1-D two-means), the paper's section 3 work count, and invariants of
Lloyd's method (fixed point, monotone J, stage handoff, translation equivariance).
"""
import itertools
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_kv(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            out[parts[0]] = parts[1] if len(parts) > 1 else None
    return out


# --------------------------------------------------------------------------- keys
def test_splitmix64_published_vector():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as f:
        rows = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    seed = int(rows[0].split()[1])
    expect = [int(v) for v in rows[1:]]
    assert [oracle.key(seed, i) for i in range(len(expect))] == expect


@pytest.mark.parametrize("n,k,f,m", [
    (100_000, 8, 0.01, 1000),        # "random 1% (1,000 points)" of the 2-D workload
    (10_000_000, 64, 0.01, 100_000),
    (100_000_000, 1024, 0.005, 500_000),
    (500_000_000, 32, 0.001, 500_000),
    (150, 2, 0.10, 15),              # Table 1: 10% of 150 points
    (1000, 4, 0.10, 100),            # section 3: N_f = 100 of N = 1000
    (10, 8, 0.01, 8),                # clamped up to k
    (10, 3, 1.0, 10),
    (7, 2, 0.5, 4),                  # floor(3.5 + 0.5)
])
def test_subset_size(n, k, f, m):
    assert oracle.subset_size(n, k, f) == m


@pytest.mark.parametrize("n,m,k,seed", [(1, 1, 1, 0), (50, 7, 3, 1), (300, 30, 5, 99),
                                        (1000, 1000, 10, 7), (2000, 13, 13, 2**63 + 5)])
def test_select_matches_full_sort(n, m, k, seed):
    keys = [(oracle.key(seed, i), i) for i in range(n)]
    order = sorted(keys)
    sub, ini = oracle.select(n, m, k, seed)
    assert sub.tolist() == sorted(i for _, i in order[:m])
    assert ini.tolist() == [i for _, i in order[:k]]
    assert set(ini.tolist()) <= set(sub.tolist())


# --------------------------------------------------------------- brute force
def _all_partitions_J(X, k):
    """J of every labeling of the rows of X into k clusters (means of non-empty ones)."""
    n, d = X.shape
    labs = np.array(list(itertools.product(range(k), repeat=n)), dtype=np.int64)
    onehot = (labs[:, :, None] == np.arange(k)[None, None, :]).astype(np.float64)
    cnt = onehot.sum(1)                                   # (L, k)
    sums = np.einsum("lik,id->lkd", onehot, X)            # (L, k, d)
    sq = (X * X).sum(1)
    tot = onehot.transpose(0, 2, 1) @ sq                  # (L, k)
    with np.errstate(invalid="ignore", divide="ignore"):
        within = np.where(cnt > 0, tot - (sums * sums).sum(2) / cnt, 0.0)
    return labs, within.sum(1), cnt


def _lloyd_stable(X, labels, centers, k):
    """Every center is the mean of its points and every point is at a nearest center."""
    for j in range(k):
        pts = X[labels == j]
        if len(pts):
            assert np.allclose(centers[j], pts.mean(0), rtol=0, atol=1e-12)
    D = ((X[:, None, :] - centers[None, :, :]) ** 2).sum(2)
    assert np.all(D[np.arange(len(X)), labels] <= D.min(1) * (1 + 1e-12) + 1e-12)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("n,k,d", [(8, 2, 2), (10, 3, 2), (12, 3, 1), (9, 2, 3)])
def test_brute_force_partitions(seed, n, k, d):
    rng = np.random.default_rng(seed * 100 + n)
    X = rng.integers(-20, 21, size=(n, d)).astype(np.float64) / 4.0
    labs, Js, cnt = _all_partitions_J(X, k)
    Jstar = Js.min()
    fit = oracle.fit(X, k, 1.0, seed, 200, 1e-300)
    assert fit.info["converged"] == [1, 1]
    _lloyd_stable(X, fit.labels, fit.centers, k)
    assert fit.info["J"] >= Jstar - 1e-9 * max(1.0, Jstar)
    # the oracle's result is one of the Lloyd-stable partitions found by enumeration
    row = np.where((labs == fit.labels[None, :]).all(1))[0]
    assert len(row) == 1 and abs(Js[row[0]] - fit.info["J"]) <= 1e-9 * max(1.0, Jstar)
    # started at the centers of an optimal partition with no empty cluster, the
    # slow stage stops after one pass with zero movement and J = J*
    full = np.where((cnt > 0).all(1))[0]
    best = full[np.argmin(Js[full])]
    C0 = np.array([X[labs[best] == j].mean(0) for j in range(k)])
    D = ((X[:, None, :] - C0[None]) ** 2).sum(2)
    if np.all(np.sort(D, 1)[:, 1] - np.sort(D, 1)[:, 0] > 1e-9) if k > 1 else True:
        f2 = oracle.fit(X, k, 1.0, seed, 50, 1e-300, init_centers=C0, skip_stage1=True)
        assert f2.info["iters"][1] == 1 and f2.info["shift"][1] == 0.0
        assert abs(f2.info["J"] - Js[best]) <= 1e-9 * max(1.0, Js[best])


def test_assign_brute_force_and_tie_rule():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(200, 5))
    C = rng.normal(size=(7, 5))
    lab, D1, D2 = oracle.assign(X, C)
    D = ((X[:, None, :] - C[None]) ** 2).sum(2)
    assert np.array_equal(lab, D.argmin(1))
    assert np.allclose(D1, D.min(1), rtol=1e-14, atol=0)
    assert np.allclose(D2, np.sort(D, 1)[:, 1], rtol=1e-14, atol=0)
    # equidistant point: the lowest center index wins; D2 == D1
    lab, D1, D2 = oracle.assign(np.zeros((1, 2)), np.array([[1.0, 0.0], [-1.0, 0.0], [0, 1.0]]))
    assert lab[0] == 0 and D1[0] == D2[0] == 1.0


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_k1_closed_form(dtype):
    rng = np.random.default_rng(11)
    X = rng.normal(3.0, 2.0, size=(5000, 3))
    if dtype == "f32":
        X = X.astype(np.float32)
    Xd = X.astype(np.float64)
    fit = oracle.fit(X, 1, 0.1, 5, 10, 1e-300)
    mean = Xd.mean(0)
    assert np.allclose(fit.centers[0], mean, rtol=1e-13, atol=1e-13)
    J = ((Xd - mean) ** 2).sum()
    assert abs(fit.info["J"] - J) <= 1e-11 * J
    # pass 1 moves the center to the stage's mean, pass 2 does not move it
    assert fit.info["iters"] == [2, 2]
    assert fit.shift_hist[0][-1] == 0.0 and fit.shift_hist[1][-1] == 0.0
    assert (fit.labels == 0).all()


def test_k_equals_n():
    rng = np.random.default_rng(2)
    X = rng.permutation(40).reshape(20, 2).astype(np.float64)  # distinct points
    fit = oracle.fit(X, 20, 1.0, 9, 5, 1e-300)
    assert fit.info["J"] == 0.0
    assert fit.info["iters"] == [1, 1]
    assert sorted(map(tuple, fit.centers)) == sorted(map(tuple, X))
    assert np.array_equal(fit.centers[fit.labels], X)


@pytest.mark.parametrize("seed", range(5))
def test_1d_two_means_contiguous_split(seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.normal(-4, 1, 300), rng.normal(5, 1.5, 200)])
    rng.shuffle(x)
    X = x[:, None]
    fit = oracle.fit(X, 2, 0.2, seed, 100, 1e-300)
    # exact optimum of 1-D two-means: the best contiguous split of the sorted data
    xs = np.sort(x)
    cs, cs2 = np.cumsum(xs), np.cumsum(xs * xs)
    n = len(xs)
    best = np.inf
    for s in range(1, n):
        l_n, r_n = s, n - s
        l_s, r_s = cs[s - 1], cs[-1] - cs[s - 1]
        J = (cs2[s - 1] - l_s ** 2 / l_n) + (cs2[-1] - cs2[s - 1] - r_s ** 2 / r_n)
        best = min(best, J)
    assert abs(fit.info["J"] - best) <= 1e-9 * best
    # the fixed point is a contiguous split at the midpoint of the two means
    lo, hi = sorted(fit.centers[:, 0])
    mid = 0.5 * (lo + hi)
    low_c = int(np.argmin(fit.centers[:, 0]))
    assert np.array_equal(fit.labels == low_c, x < mid)


# ------------------------------------------------------------------- invariants
def _mixture(seed, n=4000, d=3, k=5, spread=10.0):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-spread, spread, size=(k, d))
    comp = rng.integers(0, k, size=n)
    return (mu[comp] + rng.normal(size=(n, d))).astype(np.float32)


@pytest.mark.parametrize("seed", range(4))
def test_fixed_point_and_monotone_J(seed):
    X = _mixture(seed)
    fit = oracle.fit(X, 6, 0.1, seed, 300, 1e-300)
    assert fit.info["converged"] == [1, 1]
    _lloyd_stable(X.astype(np.float64), fit.labels, fit.centers, 6)
    for s in range(2):
        J = fit.J_hist[s]
        assert np.all(np.diff(J) <= 1e-12 * J[:-1])
        assert fit.shift_hist[s][-1] == 0.0
    # the returned J is eq. (3)'s sum at the returned centers
    D = ((X.astype(np.float64)[:, None] - fit.centers[None]) ** 2).sum(2)
    assert abs(D.min(1).sum() - fit.info["J"]) <= 1e-12 * fit.info["J"]


def _stage1_by_hand(X, k, f, seed, max_iter, tol):
    n = len(X)
    m = oracle.subset_size(n, k, f)
    sub, ini = oracle.select(n, m, k, seed)
    C = X[ini].astype(np.float64)
    Y = np.ascontiguousarray(X[sub])
    it = 0
    while it < max_iter:
        st = oracle.step(Y, C)
        C = st.C_new
        it += 1
        if st.shift < tol:
            break
    return C, it


@pytest.mark.parametrize("seed", range(3))
def test_stage_handoff(seed):
    X = _mixture(seed + 10)
    k, f, tol = 5, 0.05, 1e-6
    C1, it1 = _stage1_by_hand(X, k, f, seed, 100, tol)
    two = oracle.fit(X, k, f, seed, 100, tol)
    slow_only = oracle.fit(X, k, f, seed, 100, tol, init_centers=C1, skip_stage1=True)
    assert two.info["iters"][0] == it1
    assert np.array_equal(two.centers, slow_only.centers)
    assert np.array_equal(two.labels, slow_only.labels)
    assert two.info["iters"][1] == slow_only.info["iters"][1]
    # the slow stage's first pass runs at the fast stage's last centers
    lab, D1, _ = oracle.assign(X, C1)
    assert two.J_hist[1][0] == pytest.approx(D1.sum(), rel=1e-13)


def test_theorem_special_case_full_subset():
    """With the whole data in the fast stage, the slow stage starts at a Lloyd fixed
    point of the same data and ends after one pass that moves nothing."""
    X = _mixture(21)
    fit = oracle.fit(X, 5, 1.0, 3, 500, 1e-300)
    assert fit.info["iters"][1] == 1 and fit.info["shift"][1] == 0.0
    normal = oracle.fit(X, 5, 1.0, 3, 500, 1e-300, skip_stage1=True)
    assert np.array_equal(normal.centers, fit.centers)
    assert normal.info["iters"][1] == fit.info["iters"][0]


def test_work_count_and_section3_example():
    g = _golden_kv("complexity_section3.txt")
    K, N, Nf = int(g["K"]), int(g["N"]), int(g["N_f"])
    Qf, Qs, Q = int(g["Q_f"]), int(g["Q_s"]), int(g["Q"])
    X = _mixture(5, n=N, d=2, k=K, spread=30.0)
    # tol 0 never stops on movement, so each stage runs exactly max_iter passes
    fit = oracle.fit(X, K, Nf / N, 1, (Qf, Qs), 0.0)
    assert fit.info["m"] == Nf and fit.info["iters"] == [Qf, Qs]
    stages = fit.info["dist_evals"] - K * N  # minus the final labelling pass
    assert K * Qf * Nf == int(g["fast"]) and K * Qs * N == int(g["slow"])
    assert stages == int(g["two_stage"])
    normal = oracle.fit(X, K, Nf / N, 1, (1, Q), 0.0, skip_stage1=True)
    assert normal.info["dist_evals"] - K * N == int(g["normal"])


def test_empty_cluster_keeps_center():
    X = _mixture(8, n=500, d=2, k=3).astype(np.float64)
    C0 = np.array([X[0], X[0], [1e6, 1e6], X[1]])  # duplicate and far-away centers
    fit = oracle.fit(X, 4, 1.0, 0, 1, 0.0, init_centers=C0, skip_stage1=True)
    st = oracle.step(X, C0)
    assert st.N[1] == 0 and st.N[2] == 0 and st.empty == 2
    assert np.array_equal(st.C_new[1], C0[1]) and np.array_equal(st.C_new[2], C0[2])
    assert fit.info["empty"][1] == 2
    again = oracle.step(X, C0)
    assert np.array_equal(again.C_new, st.C_new) and np.array_equal(again.labels, st.labels)


def test_translation_equivariance():
    rng = np.random.default_rng(4)
    mu = rng.integers(-40, 40, size=(4, 3))
    X = (mu[rng.integers(0, 4, 3000)] + rng.integers(-3, 4, size=(3000, 3))).astype(np.float64)
    t = np.array([1024.0, -512.0, 256.0])
    a = oracle.fit(X, 4, 0.1, 2, 100, 1e-9)
    b = oracle.fit(X + t, 4, 0.1, 2, 100, 1e-9)
    assert np.array_equal(a.labels, b.labels)
    assert a.info["iters"] == b.info["iters"]
    assert np.allclose(b.centers - t, a.centers, rtol=0, atol=1e-9)
    assert b.info["J"] == pytest.approx(a.info["J"], rel=1e-9)


def test_bf16_input_widened_exactly():
    rng = np.random.default_rng(6)
    f = rng.normal(size=(300, 4)).astype(np.float32)
    bits = (f.view(np.uint32) >> 16).astype(np.uint16)     # truncated BF16 patterns
    wide = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    C = wide[:3].copy()
    a = oracle.step(bits, C)
    b = oracle.step(wide, C)
    assert np.array_equal(a.labels, b.labels) and a.J == b.J
    assert np.array_equal(a.C_new, b.C_new)


def test_invalid_arguments():
    X = np.zeros((5, 2))
    with pytest.raises(ValueError):
        oracle.fit(X, 6, 0.5, 0, 10, 0.0)       # k > n
    with pytest.raises(ValueError):
        oracle.fit(X, 2, 0.0, 0, 10, 0.0)       # empty subset fraction
    with pytest.raises(ValueError):
        oracle.fit(X, 2, 0.5, 0, 0, 0.0)        # no pass allowed
    with pytest.raises(ValueError):
        oracle.fit(X, 2, 0.5, 0, 10, -1.0)      # negative tolerance


def test_shift_is_euclidean_movement():
    """One pass from (0,0) to a cluster whose mean is (3,4) moves the center by 5."""
    X = np.array([[2.0, 4.0], [4.0, 4.0], [3.0, 3.0], [3.0, 5.0]])
    st = oracle.step(X, np.zeros((1, 2)))
    assert np.array_equal(st.C_new, [[3.0, 4.0]]) and st.shift == 5.0
    # largest movement over centers: second center moves by 13 (5-12-13)
    X2 = np.vstack([X, [[105.0, 112.0]]])
    st = oracle.step(X2, np.array([[0.0, 0.0], [100.0, 100.0]]))
    assert st.shift == 13.0


# ----------------------------------------------------------------- J_stage1
def test_J_stage1_is_the_last_fast_pass_before_its_update():
    """k = 1 with a tolerance so large that the fast stage stops after its
    first pass: J_stage1 is the sum over the subset of the squared distances to
    the initial center (the point with the smallest key), not to the subset's
    mean (the updated center).  Computed here from the sampled indices alone."""
    rng = np.random.default_rng(12)
    X = rng.normal(2.0, 3.0, size=(3000, 4))
    f, seed = 0.05, 17
    m = oracle.subset_size(len(X), 1, f)
    sub, ini = oracle.select(len(X), m, 1, seed)
    Y = X[sub]
    fit = oracle.fit(X, 1, f, seed, (5, 5), (1e300, 1e-300))
    assert fit.info["iters"][0] == 1
    want = ((Y - X[ini[0]]) ** 2).sum()
    assert fit.info["J_stage1"] == pytest.approx(want, rel=1e-13)
    assert abs(fit.info["J_stage1"] - ((Y - Y.mean(0)) ** 2).sum()) > 1e-3 * want
    # more passes: J_stage1 is J of the last pass, i.e. at the subset's mean
    fit = oracle.fit(X, 1, f, seed, (5, 5), 1e-300)
    assert fit.info["iters"][0] == 2
    assert fit.info["J_stage1"] == pytest.approx(((Y - Y.mean(0)) ** 2).sum(), rel=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_J_stage1_equals_hand_replay(seed):
    X = _mixture(seed + 30)
    k, f, tol = 5, 0.05, 1e-6
    n = len(X)
    sub, ini = oracle.select(n, oracle.subset_size(n, k, f), k, seed)
    Y = np.ascontiguousarray(X[sub])
    C = X[ini].astype(np.float64)
    Jlast = None
    for _ in range(100):
        st = oracle.step(Y, C)
        Jlast, C = st.J, st.C_new
        if st.shift < tol:
            break
    fit = oracle.fit(X, k, f, seed, 100, tol)
    assert fit.info["J_stage1"] == Jlast


# ------------------------------------------------------------ per-pass trace
def test_trace_hand_computed_table():
    """A Table 1 style trace worked out by hand: 1-D points 0, 1, 2, 10, 11, 12,
    two centers started at 0 and 1 (slow stage only).  Pass 1: {0} and
    {1, 2, 10, 11, 12} -> centers 0 and 7.2.  Pass 2: {0, 1, 2} and {10, 11, 12}
    -> 1 and 11.  Pass 3: the same clusters, no movement, stop."""
    X = np.array([[0.0], [1.0], [2.0], [10.0], [11.0], [12.0]])
    fit = oracle.fit(X, 2, 1.0, 0, (1, 10), (0.0, 1e-9), init_centers=np.array([[0.0], [1.0]]),
                     skip_stage1=True, trace=True)
    assert fit.info["iters"][1] == 3
    assert np.array_equal(fit.trace_centers[1][:, :, 0], [[0, 1], [0, 7.2], [1, 11]])
    assert np.array_equal(fit.trace_counts[1], [[1, 5], [3, 3], [3, 3]])
    assert np.array_equal(fit.centers[:, 0], [1, 11])


@pytest.mark.parametrize("seed", range(3))
def test_trace_rows_chain_the_passes(seed):
    """Row 0 of the fast stage holds the sampled initial centers; every later row
    holds the previous pass's new centers; the fast stage's new centers start the
    slow stage; counts are the sizes of the labels of each pass."""
    X = _mixture(seed + 40, n=3000)
    k, f, tol = 6, 0.1, 1e-6
    fit = oracle.fit(X, k, f, seed, 100, tol, trace=True)
    n = len(X)
    sub, ini = oracle.select(n, oracle.subset_size(n, k, f), k, seed)
    tc, tn = fit.trace_centers, fit.trace_counts
    assert np.array_equal(tc[0][0], X[ini].astype(np.float64))
    Ys = (np.ascontiguousarray(X[sub]), X)
    for s in range(2):
        for t in range(len(tc[s])):
            st = oracle.step(Ys[s], tc[s][t])
            assert np.array_equal(tn[s][t], np.bincount(st.labels, minlength=k))
            nxt = tc[s][t + 1] if t + 1 < len(tc[s]) else (tc[1][0] if s == 0 else fit.centers)
            assert np.array_equal(nxt, st.C_new)
    assert tn[0].sum(1).tolist() == [len(sub)] * len(tn[0])
    assert tn[1].sum(1).tolist() == [n] * len(tn[1])


# --------------------------------------------------- empty-cluster re-seeding
def test_reseed_moves_empty_center_to_farthest_point():
    """Two identical centers at 1 over the points 0, 1, 2, 100: the second one
    gets no point (lowest index on ties).  The update puts the first at the mean
    25.75; the re-seed sends the second to the point farthest from its nearest
    updated center, 100 (distance 74.25 to 25.75), a movement of 99."""
    X = np.array([[0.0], [1.0], [2.0], [100.0]])
    C = np.array([[1.0], [1.0]])
    keep = oracle.step(X, C)
    assert keep.empty == 1 and np.array_equal(keep.C_new[:, 0], [25.75, 1.0])
    assert keep.shift == 24.75
    re = oracle.step(X, C, reseed=True)
    assert re.empty == 1 and np.array_equal(re.N, [4, 0])
    assert np.array_equal(re.C_new[:, 0], [25.75, 100.0]) and re.shift == 99.0
    assert np.array_equal(re.labels, keep.labels) and re.J == keep.J


def test_reseed_tie_goes_to_lowest_point_and_one_cluster_per_pass():
    """Points -10, 0, 10 and three centers at 0: clusters 1 and 2 are empty; only
    cluster 1 is re-seeded, to -10 (as far as 10 from the updated center 0, and
    first); cluster 2 keeps its center until a later pass."""
    X = np.array([[-10.0], [0.0], [10.0]])
    st = oracle.step(X, np.zeros((3, 1)), reseed=True)
    assert st.empty == 2
    assert np.array_equal(st.C_new[:, 0], [0.0, -10.0, 0.0]) and st.shift == 10.0
    st2 = oracle.step(X, st.C_new, reseed=True)
    # next pass from 0, -10, 0: -10 joins cluster 1; 0 and 10 go to cluster 0
    # (ties with cluster 2), whose mean is 5; cluster 2 is empty and takes the
    # point farthest from its nearest of 5, -10, 0: 10 (at 5 from 5)
    assert np.array_equal(st2.N, [2, 1, 0]) and st2.empty == 1
    assert np.array_equal(st2.C_new[:, 0], [5.0, -10.0, 10.0])


def test_reseed_fit_ends_without_empty_clusters():
    """Two starting centers far outside the data never win a point under the
    keep rule; with re-seeding (one per pass) every cluster ends with members
    and J is lower."""
    X = _mixture(50, n=2000, d=2, k=4, spread=20.0).astype(np.float64)
    C0 = np.array([X[0], X[1], [1e6, 1e6], [-1e6, 1e6]])
    keep = oracle.fit(X, 4, 1.0, 0, (1, 100), 1e-9, init_centers=C0, skip_stage1=True)
    re = oracle.fit(X, 4, 1.0, 0, (1, 100), 1e-9, init_centers=C0, skip_stage1=True, reseed=True)
    assert keep.info["empty"][1] == 2
    assert re.info["empty"][1] == 0 and re.info["converged"][1] == 1
    assert re.info["J"] < keep.info["J"]
    _lloyd_stable(X, re.labels, re.centers, 4)
