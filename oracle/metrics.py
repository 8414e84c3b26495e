"""Error measures of an emulated product against a double-double reference.

TEST INFRASTRUCTURE ONLY.

err_comp (the accuracy gate): max_ij |C_hat - C*|_ij / (|op(A)| |op(B)|)_ij,
with |.| the complex modulus entrywise. It is unchanged by power-of-two scaling
of rows of A or columns of B and is the quantity the slicing error bound
controls. The paper reports a percent error of its application output against
native FP64 (Section 3.2) and fixes no GEMM-level measure; this is the reading
used throughout. An entry with a zero denominator must be exactly zero.

err_norm = max |C_hat - C*| / max |C*|;  err_elem = max |C_hat - C*|_ij / |C*_ij|
(both reported for information only; err_elem is unbounded under cancellation).
"""
from __future__ import annotations

import numpy as np

from .ozaki import op


def _diff(C_hat, hi, lo):
    # (C_hat - hi) is exact when C_hat is close to hi (Sterbenz); subtracting lo
    # then rounds once.
    return np.abs((C_hat - hi) - lo)


def abs_product(transa, transb, A, B):
    """(|op(A)| |op(B)|) in FP64 (entrywise moduli)."""
    return np.abs(op(np.asarray(A), transa)) @ np.abs(op(np.asarray(B), transb))


def err_comp(C_hat, hi, lo, denom) -> float:
    d = _diff(np.asarray(C_hat), hi, lo)
    den = np.asarray(denom, dtype=np.float64)
    zero = den == 0
    if np.any(d[zero] != 0):
        return float("inf")
    if np.any(~np.isfinite(d[~zero])):
        return float("inf")
    r = np.zeros_like(d, dtype=np.float64)
    r[~zero] = d[~zero] / den[~zero]
    return float(r.max()) if r.size else 0.0


def err_norm(C_hat, hi, lo) -> float:
    d = _diff(np.asarray(C_hat), hi, lo)
    ref = np.abs(hi)
    mx = ref.max() if ref.size else 0.0
    return float(d.max() / mx) if mx > 0 else float(d.max() if d.size else 0.0)


def err_elem(C_hat, hi, lo) -> float:
    d = _diff(np.asarray(C_hat), hi, lo)
    ref = np.abs(hi)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(ref > 0, d / ref, np.where(d == 0, 0.0, np.inf))
    return float(r.max()) if r.size else 0.0


def denom_entries(transa, transb, A, B, rows, cols):
    """(|op(A)| |op(B)|) at selected entries only."""
    opA = np.abs(op(np.asarray(A), transa))
    opB = np.abs(op(np.asarray(B), transb))
    return np.einsum("xl,lx->x", opA[np.asarray(rows)], opB[:, np.asarray(cols)])
