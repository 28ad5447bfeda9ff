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
