"""Batched fits and the serving loop against the FP64 oracle, through the C ABI.

kmeans_fit_batch advances many independent two-stage fits in shared launches;
each problem must still match the oracle run on its own data (iterations,
centers, J, labels).  The server admits problems by device-memory footprint
and batches their passes as they arrive; a problem's result must be the same
bits alone and in a mix.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import JTOL, assert_centers, assert_labels, j_atol, to_device

pytestmark = pytest.mark.gpu

km = pytest.importorskip("paper_1108_1351_amd")


def _problem(n, d, k, seed, dtype):
    spec = synth.MixtureSpec(d, max(2, k // 2), "uniform", -15.0, 15.0, sigma_lo=0.5,
                             sigma_hi=2.0, weights="dirichlet1")
    return synth.generate(spec, seed, n, dtype)


# (n, d, k, dtype, subset_frac, seed, max_iter, tol)
PROBLEMS = [
    (3_000, 2, 4, "f32", 0.05, 1, (30, 30), (1e-4, 1e-4)),
    (20_011, 8, 16, "f32", 0.02, 2, (20, 25), (1e-3, 1e-5)),
    (1_000, 3, 7, "f32", 0.5, 3, (40, 40), (0.0, 0.0)),
    (5_003, 32, 64, "bf16", 0.1, 4, (10, 10), (1e-4, 1e-4)),
    (12_000, 128, 100, "bf16", 0.05, 5, (6, 8), (1e-4, 1e-4)),
    (40_000, 16, 256, "f32", 0.01, 6, (8, 8), (1e-4, 1e-4)),   # sums beyond LDS: k_batch_sums
    (700, 64, 9, "f32", 1.0, 7, (15, 15), (1e-6, 1e-6)),
    (15_000, 64, 100, "f32", 0.05, 8, (6, 6), (1e-4, 1e-4)),   # k_batch_sums, whole pieces
    (9_001, 37, 220, "f32", 0.05, 9, (5, 5), (1e-4, 1e-4)),    # k_batch_sums, element loads
    (30_000, 128, 200, "bf16", 0.02, 10, (4, 6), (1e-4, 1e-4)),  # four center ranges
]


def _check_against_oracle(Xh, C, L, info, k, f, seed, mi, tl, name):
    ref = oracle.fit(Xh, k, f, seed, mi, tl)
    assert info["status"] == 0, name
    assert info["m"] == ref.info["m"], name
    assert info["iters"] == ref.info["iters"], (name, info["iters"], ref.info["iters"])
    assert info["converged"] == ref.info["converged"], name
    assert info["dist_evals"] == ref.info["dist_evals"], name
    assert_centers(C.cpu().numpy().astype(np.float64), ref.centers, Xh, tol=1e-5, name=name)
    assert abs(info["J"] - ref.info["J"]) <= JTOL * ref.info["J"] + j_atol(Xh), name
    assert abs(info["J_stage1"] - ref.info["J_stage1"]) <= JTOL * ref.info["J_stage1"] + j_atol(Xh)
    assert_labels(L, Xh, ref.centers, ref_labels=ref.labels, name=name)


def test_fit_batch_matches_oracle_per_problem():
    data = [_problem(n, d, k, 100 + s, dt) for (n, d, k, dt, f, s, mi, tl) in PROBLEMS]
    probs = [(to_device(Xh), k, f, s, mi, tl)
             for Xh, (n, d, k, dt, f, s, mi, tl) in zip(data, PROBLEMS)]
    print(f"[batch] {len(probs)} problems", flush=True)
    out = km.kmeans_fit_batch(probs)
    for Xh, (C, L, info), (n, d, k, dt, f, s, mi, tl) in zip(data, out, PROBLEMS):
        _check_against_oracle(Xh, C, L, info, k, f, s, mi, tl, f"n={n} d={d} k={k} {dt}")


def test_fit_batch_one_bad_problem_others_complete():
    Xa = _problem(2_000, 4, 5, 11, "f32")
    Xb = _problem(50, 4, 5, 12, "f32")
    probs = [(to_device(Xa), 5, 0.1, 1, 20, 1e-4), (to_device(Xb), 60, 0.5, 1, 20, 1e-4)]
    out = km.kmeans_fit_batch(probs)
    assert out[1][2]["status"] == km.KM_EINVAL
    _check_against_oracle(Xa, out[0][0], out[0][1], out[0][2], 5, 0.1, 1, (20, 20),
                          (1e-4, 1e-4), "good problem")


def test_fit_batch_many_small_problems():
    rng = np.random.default_rng(9)
    specs = []
    for i in range(40):
        n = int(rng.integers(300, 4000))
        d = int(rng.choice([2, 8, 32]))
        k = int(rng.integers(2, 24))
        specs.append((n, d, k, "f32" if d < 32 else "bf16", 0.2, 1000 + i, (15, 15),
                      (1e-4, 1e-4)))
    data = [_problem(n, d, k, s, dt) for (n, d, k, dt, f, s, mi, tl) in specs]
    out = km.kmeans_fit_batch([(to_device(Xh), k, f, s, mi, tl)
                               for Xh, (n, d, k, dt, f, s, mi, tl) in zip(data, specs)])
    for Xh, (C, L, info), (n, d, k, dt, f, s, mi, tl) in zip(data, out, specs):
        _check_against_oracle(Xh, C, L, info, k, f, s, mi, tl, f"n={n} d={d} k={k}")


def test_tune_query_returns_a_valid_tile():
    for d, k in [(2, 8), (8, 100), (32, 256), (128, 64)]:
        ppt, kt = km.km_tune_query(torch.float32, d, k)
        assert ppt in (1, 2, 4) and kt in (32, 64, 128, 256)


def _serve_one(srv, Xh, k, f, seed, mi, tl):
    t = srv.submit(torch.from_numpy(Xh.view(np.int16) if Xh.dtype == np.uint16 else Xh)
                   .view(torch.bfloat16 if Xh.dtype == np.uint16 else torch.float32),
                   k, f, seed, mi, tl)
    return t


def test_server_result_same_alone_and_in_mix():
    target = (_problem(30_000, 8, 24, 77, "f32"), 24, 0.02, 5, (25, 25), (1e-4, 1e-4))
    Xh, k, f, seed, mi, tl = target
    with km.Server() as srv:
        t = _serve_one(srv, Xh, k, f, seed, mi, tl)
        C0, L0, info0 = srv.wait(t, timeout=120)
    rng = np.random.default_rng(3)
    others = [(_problem(int(rng.integers(500, 20000)), int(d), int(rng.integers(3, 40)), 500 + i,
                        "f32" if d < 32 else "bf16"))
              for i, d in enumerate(rng.choice([2, 8, 32, 128], size=24))]
    with km.Server() as srv:
        tickets = []
        for i, Xo in enumerate(others[:12]):
            tickets.append(_serve_one(srv, Xo, min(16, len(Xo) // 10), 0.1, i, (10, 10),
                                      (1e-4, 1e-4)))
        t = _serve_one(srv, Xh, k, f, seed, mi, tl)
        for i, Xo in enumerate(others[12:]):
            tickets.append(_serve_one(srv, Xo, min(16, len(Xo) // 10), 0.1, 12 + i, (10, 10),
                                      (1e-4, 1e-4)))
        C1, L1, info1 = srv.wait(t, timeout=120)
        for tt in tickets:
            srv.wait(tt, timeout=120)
        st = srv.stats()
    assert st["completed"] == 25 and st["failed"] == 0
    assert torch.equal(C0, C1)
    assert torch.equal(L0, L1)
    assert info0["J"] == info1["J"] and info0["iters"] == info1["iters"]
    _check_against_oracle(Xh, C1, L1, info1, k, f, seed, mi, tl, "served")


@pytest.mark.parametrize("d,k,comps", [(128, 64, 8), (32, 200, 20), (100, 40, 4)])
def test_fit_batch_bf16_screen_tight_clusters_far_out(d, k, comps):
    """Tight components far from the origin with several centers each: many
    points have three or more centers inside the screen's error band, so the
    candidate lists (and, beyond them, the FP64 check over all centers) decide."""
    spec = synth.MixtureSpec(d, comps, "uniform", -50.0, 50.0, sigma_lo=0.5, sigma_hi=0.5,
                             weights="dirichlet1")
    Xh = synth.generate(spec, 4321 + d, 12_000, "bf16")
    X = torch.from_numpy(Xh.view(np.int16)).cuda().view(torch.bfloat16)
    mi, tl = (5, 8), (0.0, 0.0)
    (C, L, info), = km.kmeans_fit_batch([(X, k, 0.05, 7, mi, tl)])
    _check_against_oracle(Xh, C, L, info, k, 0.05, 7, mi, tl, f"tight {d} {k}")


def test_server_pass_chunks_same_results():
    """Chunks of passes between host synchronisations change nothing but the
    number of synchronisations: problems that stop early (tol) inside a chunk are
    skipped by the device until it ends."""
    rng = np.random.default_rng(11)
    probs = [(_problem(int(rng.integers(2_000, 30_000)), int(d), int(rng.integers(4, 40)), 700 + i,
                       "f32" if d < 32 else "bf16"))
             for i, d in enumerate(rng.choice([3, 8, 16, 64, 128], size=16))]
    out = {}
    for pps in (1, 8):
        with km.Server(passes_per_sync=pps) as srv:
            ts = [_serve_one(srv, Xh, min(24, len(Xh) // 50), 0.05, i, (20, 30), (1e-3, 1e-4))
                  for i, Xh in enumerate(probs)]
            out[pps] = [srv.wait(t, timeout=120) for t in ts]
            out[pps, "st"] = srv.stats()
    for i in range(len(probs)):
        C1, L1, i1 = out[1][i]
        C8, L8, i8 = out[8][i]
        assert torch.equal(C1, C8) and torch.equal(L1, L8), i
        assert i1["iters"] == i8["iters"] and i1["J"] == i8["J"], i
    assert out[8, "st"]["syncs"] < out[1, "st"]["syncs"]
    assert out[1, "st"]["syncs"] == out[1, "st"]["rounds"]
    Xh = probs[0]
    _check_against_oracle(Xh, *out[8][0], min(24, len(Xh) // 50), 0.05, 0, (20, 30), (1e-3, 1e-4),
                          "chunked")


def test_server_admission_respects_budget():
    probs = [(_problem(20_000, 8, 8, 900 + i, "f32"), 8) for i in range(6)]
    with km.Server() as probe:
        t = _serve_one(probe, probs[0][0], 8, 0.1, 0, 10, 1e-4)
        probe.wait(t, timeout=60)
        one = probe.stats()["peak_bytes"]
    budget = int(one * 2.5)  # room for two problems at a time
    with km.Server(hbm_budget_bytes=budget) as srv:
        ts = [_serve_one(srv, Xh, k, 0.1, i, 10, 1e-4) for i, (Xh, k) in enumerate(probs)]
        res = [srv.wait(t, timeout=120) for t in ts]
        st = srv.stats()
    assert st["completed"] == 6
    assert st["peak_bytes"] <= budget
    assert st["peak_active"] <= 2
    for (Xh, k), (C, L, info), i in zip(probs, res, range(6)):
        _check_against_oracle(Xh, C, L, info, k, 0.1, i, (10, 10), (1e-4, 1e-4), f"budget {i}")


def test_server_rejects_bad_request_and_unknown_ticket():
    with km.Server() as srv:
        with pytest.raises(km.KMeansError) as e:
            srv.submit(torch.zeros((10, 4)), 20, 0.5, 0)
        assert e.value.status == km.KM_EINVAL
        res = km.km_result()
        rc = km.load().km_server_wait(srv._h, 12345, res, 0)
        assert rc == km.KM_ENOTFOUND


def test_server_over_budget_submit_is_enomem():
    with km.Server(hbm_budget_bytes=1 << 20) as srv:
        with pytest.raises(km.KMeansError) as e:
            srv.submit(torch.from_numpy(_problem(200_000, 8, 8, 1, "f32")), 8, 0.1, 0)
        assert e.value.status == km.KM_ENOMEM
        assert srv.stats()["submitted"] == 0


def test_server_destroy_with_jobs_in_flight_and_blocked_waiter():
    """Destroy while problems run and wait, with another thread blocked in
    km_server_wait: destroy returns, the waiter returns KM_ECANCELLED (or its
    result, had it finished first), and nothing else happens to the process."""
    import threading

    Xs = [_problem(200_000, 32, 64, 300 + i, "f32") for i in range(6)]
    # room for two problems at a time: four wait in the queue; thousands of
    # passes each (tol 0) keep the two admitted ones running
    srv = km.Server(hbm_budget_bytes=70 << 20)
    tickets = [srv.submit(torch.from_numpy(X), 64, 0.05, i, (2000, 4000), (0.0, 0.0))
               for i, X in enumerate(Xs)]
    outcome = {}

    def waiter():
        try:
            srv.wait(tickets[-1])
            outcome["status"] = km.KM_OK
        except km.KMeansError as e:
            outcome["status"] = e.status

    th = threading.Thread(target=waiter)
    th.start()
    import time
    time.sleep(1.0)  # the waiter is inside km_server_wait by now
    st = srv.stats()
    assert st["pending"] + st["active"] > 0
    srv.close()  # km_server_destroy
    th.join(timeout=60)
    assert not th.is_alive()
    assert outcome["status"] in (km.KM_OK, km.KM_ECANCELLED)
    # the device is still usable
    Xh = _problem(2_000, 4, 5, 11, "f32")
    _check_against_oracle(Xh, *km.kmeans_fit_batch([(to_device(Xh), 5, 0.1, 1, 20, 1e-4)])[0],
                          5, 0.1, 1, (20, 20), (1e-4, 1e-4), "after destroy")


def test_server_bf16_128d_target_same_alone_and_in_mix():
    """A 128-D BF16 request (the batched BF16 MFMA screen) gives the same bits
    alone and among other requests of every shape, and matches the oracle."""
    target = (_problem(40_000, 128, 48, 91, "bf16"), 48, 0.02, 6, (20, 20), (1e-4, 1e-4))
    Xh, k, f, seed, mi, tl = target
    with km.Server() as srv:
        t = _serve_one(srv, Xh, k, f, seed, mi, tl)
        C0, L0, info0 = srv.wait(t, timeout=120)
    rng = np.random.default_rng(8)
    others = [(_problem(int(rng.integers(500, 30000)), int(d), int(rng.integers(3, 40)),
                        700 + i, "f32" if d < 32 else "bf16"))
              for i, d in enumerate(rng.choice([2, 8, 32, 64, 128], size=20))]
    with km.Server() as srv:
        tickets = [_serve_one(srv, Xo, min(32, len(Xo) // 10), 0.1, i, (10, 10), (1e-4, 1e-4))
                   for i, Xo in enumerate(others[:10])]
        t = _serve_one(srv, Xh, k, f, seed, mi, tl)
        tickets += [_serve_one(srv, Xo, min(32, len(Xo) // 10), 0.1, 10 + i, (10, 10),
                               (1e-4, 1e-4)) for i, Xo in enumerate(others[10:])]
        C1, L1, info1 = srv.wait(t, timeout=120)
        for tt in tickets:
            srv.wait(tt, timeout=120)
    assert torch.equal(C0, C1) and torch.equal(L0, L1)
    assert info0["J"] == info1["J"] and info0["iters"] == info1["iters"]
    _check_against_oracle(Xh, C1, L1, info1, k, f, seed, mi, tl, "served 128-D BF16")


@pytest.mark.parametrize("d,k", [(32, 7), (64, 33), (128, 256), (100, 65), (24, 3)])
def test_fit_batch_bf16_screen_shapes(d, k):
    """The batched BF16 screen over its shapes: 2, 4 or 8 K steps, partial last
    center tile, k up to 256, d not a multiple of 16, ragged last unit."""
    n = 9_001
    Xh = _problem(n, d, max(2, k // 2), 40 + d + k, "bf16")
    out = km.kmeans_fit_batch([(to_device(Xh), k, 0.2, 3, (8, 8), (1e-5, 1e-5))])
    C, L, info = out[0]
    _check_against_oracle(Xh, C, L, info, k, 0.2, 3, (8, 8), (1e-5, 1e-5), f"d={d} k={k}")
