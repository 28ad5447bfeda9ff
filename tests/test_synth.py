"""The seeded input generator: chunk invariance, distribution moments, rounding."""
import math

import numpy as np
import pytest

import synth


def test_chunked_equals_whole():
    spec = synth.MixtureSpec(5, 7, "uniform", -3, 3, sigma_lo=0.5, sigma_hi=2.0,
                             weights="dirichlet1")
    whole, comp = synth.generate(spec, 42, 10_001, with_comp=True)
    parts = [synth.generate(spec, 42, m, row0=r0) for r0, m in
             ((0, 3), (3, 4998), (5001, 5000))]
    assert np.array_equal(np.concatenate(parts), whole)
    assert comp.min() >= 0 and comp.max() < 7


def test_uniform_and_normal_moments():
    u = np.array([synth.uniform(9, 3, i) for i in range(20000)])
    assert 0.0 < u.min() and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1 / 12) < 0.003
    z = np.array([synth.normal(9, 4, i) for i in range(20000)])
    assert abs(z.mean()) < 0.03 and abs(z.var() - 1.0) < 0.04
    assert abs(np.mean(z ** 4) - 3.0) < 0.2  # Gaussian kurtosis


def test_mixture_structure():
    spec = synth.MixtureSpec(3, 4, "uniform", -50, 50, sigma_lo=0.5, sigma_hi=2.0,
                             weights="dirichlet1")
    means, sig, cumw = synth.params(spec, 7)
    assert np.all((-50 <= means) & (means <= 50)) and np.all((0.5 <= sig) & (sig <= 2.0))
    assert np.all(np.diff(cumw) > 0) and cumw[-1] == 1.0
    X, comp = synth.generate(spec, 7, 200_000, dtype="f64", with_comp=True)
    w = np.diff(np.concatenate([[0.0], cumw]))
    freq = np.bincount(comp, minlength=4) / len(comp)
    assert np.allclose(freq, w, atol=0.005)
    for c in range(4):
        Z = (X[comp == c] - means[c]) / sig[c]
        assert np.allclose(Z.mean(0), 0.0, atol=0.03)
        assert np.allclose(Z.std(0), 1.0, atol=0.03)


def test_normal_means_spec():
    spec = synth.MixtureSpec(128, 1024, "normal", mean_sd=5.0, sigma_lo=0.5, sigma_hi=1.5)
    means, sig, cumw = synth.params(spec, 1003)
    assert abs(means.mean()) < 0.05 and abs(means.std() - 5.0) < 0.05
    assert np.allclose(np.diff(np.concatenate([[0.0], cumw])), 1 / 1024)


def test_bf16_is_nearest_even_of_f64():
    spec = synth.MixtureSpec(4, 3, "normal", mean_sd=5.0, sigma_lo=0.5, sigma_hi=1.5)
    x64 = synth.generate(spec, 3, 20000, dtype="f64")
    b = synth.generate(spec, 3, 20000, dtype="bf16")
    f = synth.bf16_to_f32(b).astype(np.float64)
    # neighbours of the chosen BF16 value one unit away on each side
    bits = b.astype(np.int64)
    up = synth.bf16_to_f32((bits + 1).astype(np.uint16)).astype(np.float64)
    dn = synth.bf16_to_f32((bits - 1).astype(np.uint16)).astype(np.float64)
    err = np.abs(f - x64)
    assert np.all(err <= np.abs(up - x64)) and np.all(err <= np.abs(dn - x64))
    x32 = synth.generate(spec, 3, 20000, dtype="f32")
    assert np.array_equal(x32, x64.astype(np.float32))


def test_workload_table():
    w = synth.WORKLOADS["gmm2d_n1e5_k8"]
    assert (w.n, w.d, w.k, w.subset_frac, w.max_iter, w.tol) == (100_000, 2, 8, 0.01, 100, 1e-4)
    w = synth.WORKLOADS["gmm4d_n5e8_k32"]
    assert w.n * w.d * 4 == 8_000_000_000  # 8 GB of FP32 points
    reqs = synth.serving_stream(200, 50.0)
    t = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() * 50.0 - 1.0) < 0.2
    ns = np.array([r.workload.n for r in reqs])
    assert ns.min() >= 1000 and ns.max() <= 1_000_000
    assert {r.workload.d for r in reqs} == {2, 8, 32, 128}
    assert all(4 <= r.workload.k <= 256 for r in reqs)
    assert math.isclose(np.log10(ns).mean(), 4.5, abs_tol=0.25)
