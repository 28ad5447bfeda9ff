"""Shared helpers of the GPU parity tests (comparison rules against the oracle)."""
import numpy as np
import torch

import oracle

# Tolerances of the parity protocol: labels identical except where the oracle's
# top-2 relative gap (D2 - D1) / D2 is below GAP; centers within CTOL relative
# to max(||c||, rms row norm); J within JTOL relative, plus JABS * sum ||x||^2
# absolute (a floor for fits whose J is zero: the sorted update rounds each
# point's squared distance to units far below that).
GAP = 1e-6
CTOL = 1e-5
JTOL = 1e-6
JABS = 1e-12


def j_atol(Xh) -> float:
    X = widen(Xh)
    return JABS * float((X * X).sum())


def to_device(Xh: np.ndarray) -> torch.Tensor:
    if Xh.dtype == np.uint16:  # BF16 bit patterns
        return torch.from_numpy(Xh.view(np.int16)).to("cuda").view(torch.bfloat16)
    return torch.from_numpy(Xh).to("cuda")


def exempt_mask(Xh, C):
    _, D1, D2 = oracle.assign(Xh, C)
    return (D2 - D1) < GAP * D2


def assert_labels(gpu_labels, Xh, C_ref, ref_labels=None, name=""):
    """GPU labels equal the FP64 nearest centers of C_ref except at near-ties.
    Returns the number of exempt points."""
    lab = gpu_labels.cpu().numpy() if hasattr(gpu_labels, "cpu") else gpu_labels
    if ref_labels is None:
        ref_labels, D1, D2 = oracle.assign(Xh, C_ref)
    else:
        _, D1, D2 = oracle.assign(Xh, C_ref)
    ex = (D2 - D1) < GAP * D2
    bad = np.where((lab != ref_labels) & ~ex)[0]
    assert len(bad) == 0, f"{name}: {len(bad)} label mismatches, first rows {bad[:5]}"
    return int(ex.sum())


def row_scale(Xh):
    X = Xh.astype(np.float64) if Xh.dtype != np.uint16 else \
        (Xh.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return float(np.sqrt((X * X).sum(1).mean()))


def assert_centers(C_gpu, C_ref, Xh, tol=CTOL, name=""):
    scale = np.maximum(np.linalg.norm(C_ref, axis=1), row_scale(Xh))
    err = np.linalg.norm(C_gpu - C_ref, axis=1) / scale
    assert err.max() <= tol, f"{name}: center error {err.max():.3e}"
    return float(err.max())


def widen(Xh):
    if Xh.dtype == np.uint16:
        return (Xh.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return Xh.astype(np.float64)


def sums_from_labels(Xh, lab, k):
    """FP64 cluster sums, sums of |x| and counts of the rows of X under the given
    labels (bincount with weights: sums in row order)."""
    X = widen(Xh)
    d = X.shape[1]
    N = np.bincount(lab, minlength=k).astype(np.int64)
    S = np.empty((k, d))
    A = np.empty((k, d))
    for t in range(d):
        S[:, t] = np.bincount(lab, weights=X[:, t], minlength=k)
        A[:, t] = np.bincount(lab, weights=np.abs(X[:, t]), minlength=k)
    return S, A, N


def assert_step(out, Xh, C, ref, ctol=1e-9, jtol=1e-12, name=""):
    """One pass of the GPU against the oracle's pass at the same centers.

    Labels equal the oracle's except at near-ties (the GPU may pick either
    center there).  Counts, sums, new centers, movement and empties are then
    checked unconditionally against FP64 sums built from the GPU's own labels
    (and, when no label differs, against the oracle's directly): counts exactly,
    sums within the fixed-point quantum (|x| 2^F < 2^30 per term), new centers
    within ctol.  J within jtol of the oracle's J, or of the J of the GPU's
    labels when near-tie labels differ."""
    lab = out["labels"].cpu().numpy()
    k, d = C.shape
    ex = exempt_mask(Xh, C)
    bad = np.where((lab != ref.labels) & ~ex)[0]
    assert len(bad) == 0, f"{name}: {len(bad)} label mismatches, first rows {bad[:5]}"
    X = widen(Xh)
    same = bool(np.array_equal(lab, ref.labels))
    if "N" in out:
        S_l, A_l, N_l = sums_from_labels(Xh, lab, k)
        assert np.array_equal(out["N"].cpu().numpy(), N_l), name
        amax = np.abs(X).max() if X.size else 0.0
        quantum = 2.0 ** (np.floor(np.log2(amax)) - 29) if amax > 0 else 0.0
        S = out["S"].cpu().numpy()
        assert np.all(np.abs(S - S_l) <= N_l[:, None] * quantum + 1e-12 * A_l), name
        C_exp = np.where(N_l[:, None] > 0, S_l / np.maximum(N_l, 1)[:, None], C)
        assert_centers(out["C_new"].cpu().numpy(), C_exp, Xh, tol=ctol, name=name + " C_new")
        sh = float(np.sqrt(((C_exp - C) ** 2).sum(1)).max())
        assert abs(out["shift"] - sh) <= ctol * max(1.0, sh) * 10, name
        assert out["empty"] == int((N_l == 0).sum()), name
        if same:
            assert np.array_equal(out["N"].cpu().numpy(), ref.N), name
            assert_centers(out["C_new"].cpu().numpy(), ref.C_new, Xh, tol=ctol, name=name)
            assert out["empty"] == ref.empty, name
    Jref = ref.J if same else float(((X - C[lab]) ** 2).sum())
    assert abs(out["J"] - Jref) <= jtol * max(Jref, 1e-300), (name, out["J"], Jref)
    return int(ex.sum())
