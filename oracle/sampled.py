"""Accuracy of a large product on sampled entries: double-double values and
componentwise denominators of a set of output entries that the oracle can
afford one by one.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A full double-double product of 16384^3 complex operands is 1.8e13 dd
multiply-adds; the error measure err_comp (oracle.metrics) is a maximum over
entries, so a large product is judged on a sample of its entries instead:
`nrand` entries drawn uniformly, plus `nrows` whole rows and `ncols` whole
columns of C (the rows hold every column exponent f_j and the columns every
row exponent e_i, so each scaling of the operands appears at least once).

Callers that already hold op(B)^T contiguously (a column-major device copy of
B read back to the host, for instance) pass it as `Bt` to avoid a 4 GiB
transposing copy.
"""
from __future__ import annotations

import numpy as np

from . import dd, metrics


def sample_entries(m: int, n: int, nrand: int = 4096, nrows: int = 4, ncols: int = 4,
                   seed: int = 2024):
    """Output entries (ri, cj) to check: nrand uniform draws, then every entry
    of nrows rows and of ncols columns (the last row and column of C are among
    them whenever rows or columns are asked for, so the ragged edge tiles are
    covered; nrows >= m takes every row)."""
    rng = np.random.default_rng(seed)
    ri = [rng.integers(0, m, nrand)]
    cj = [rng.integers(0, n, nrand)]
    def pick(total, cnt):
        if cnt >= total:
            return np.arange(total, dtype=np.int64)
        if cnt <= 0:
            return np.zeros(0, dtype=np.int64)
        return np.unique(np.concatenate([rng.choice(total - 1, cnt - 1, replace=False),
                                         [total - 1]]))

    rows = pick(m, nrows)
    cols = pick(n, ncols)
    for r in rows:
        ri.append(np.full(n, r, dtype=np.int64))
        cj.append(np.arange(n, dtype=np.int64))
    for c in cols:
        ri.append(np.arange(m, dtype=np.int64))
        cj.append(np.full(m, c, dtype=np.int64))
    return (np.concatenate(ri).astype(np.int64), np.concatenate(cj).astype(np.int64),
            rows.astype(np.int64), cols.astype(np.int64))


def denominators(A: np.ndarray, Bt: np.ndarray, ri, cj, rows, cols) -> np.ndarray:
    """(|op(A)| |op(B)|) at the entries (ri, cj) made by sample_entries; A is
    op(A) (m x k), Bt is op(B)^T (n x k). Whole rows and columns are formed as
    matrix-vector products; the remaining entries one by one."""
    m, n = A.shape[0], Bt.shape[0]
    den = np.empty(ri.size, dtype=np.float64)
    nrand = ri.size - rows.size * n - cols.size * m
    absBt = None
    for x in range(0, nrand, 256):
        sl = slice(x, min(nrand, x + 256))
        den[sl] = np.einsum("xl,xl->x", np.abs(A[ri[sl]]), np.abs(Bt[cj[sl]]))
    off = nrand
    if rows.size:
        absBt = np.abs(Bt)
        for r in rows:
            den[off:off + n] = absBt @ np.abs(A[r])
            off += n
        del absBt
    if cols.size:
        absA = np.abs(A)
        for c in cols:
            den[off:off + m] = absA @ np.abs(Bt[c])
            off += m
        del absA
    return den


class SampledReference:
    """dd reference values and denominators of sampled entries of op(A) op(B)
    (transa = transb = 'N'); err_comp(C_at_entries) is then the componentwise
    error of a candidate product on those entries."""

    def __init__(self, A: np.ndarray, B: np.ndarray | None = None, Bt: np.ndarray | None = None,
                 nrand: int = 4096, nrows: int = 4, ncols: int = 4, seed: int = 2024):
        if Bt is None:
            Bt = np.ascontiguousarray(np.asarray(B).T)
        A = np.ascontiguousarray(A)
        m, n = A.shape[0], Bt.shape[0]
        self.ri, self.cj, self.rows, self.cols = sample_entries(m, n, nrand, nrows, ncols, seed)
        # dd_entries forms op(B)^T = B.T; handing it Bt.T makes that a view of Bt
        self.hi, self.lo = dd.dd_entries("N", "N", A, Bt.T, self.ri, self.cj)
        self.den = denominators(A, Bt, self.ri, self.cj, self.rows, self.cols)

    @property
    def count(self) -> int:
        return int(self.ri.size)

    def err_comp(self, C_at_entries) -> float:
        return metrics.err_comp(np.asarray(C_at_entries), self.hi, self.lo, self.den)
