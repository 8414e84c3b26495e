"""Helpers of the GPU tests: column-major device buffers from numpy arrays and
back, and bitwise comparisons. Host logic only."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(X: np.ndarray):
    """Column-major device copy of the matrix X; returns (tensor, ld)."""
    X = np.asarray(X)
    dt = torch.complex128 if np.iscomplexobj(X) else torch.float64
    t = torch.from_numpy(np.ascontiguousarray(X.T)).to(dtype=dt).cuda()
    return t, max(1, X.shape[0])


def host(t, rows: int, cols: int) -> np.ndarray:
    """Matrix (rows x cols) from a column-major device buffer made by dev()."""
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return np.ascontiguousarray(a.reshape(cols, rows).T)


def bits_equal(x, y) -> bool:
    """Bitwise equality of float64/complex128 arrays; NaN equals NaN."""
    x = np.ascontiguousarray(np.asarray(x))
    y = np.ascontiguousarray(np.asarray(y))
    if x.shape != y.shape or x.dtype != y.dtype:
        return False
    xn, yn = np.isnan(x), np.isnan(y)
    if not np.array_equal(xn, yn):
        return False
    xb = np.where(xn, 0, x).view(np.uint64)
    yb = np.where(yn, 0, y).view(np.uint64)
    return np.array_equal(xb, yb)


def mismatch_report(x, y, limit=5) -> str:
    x = np.asarray(x)
    y = np.asarray(y)
    bad = np.argwhere(~((x == y) | (np.isnan(x) & np.isnan(y))))
    lines = [f"{len(bad)} mismatches of {x.size}"]
    for idx in bad[:limit]:
        lines.append(f"  {tuple(idx)}: gpu={x[tuple(idx)]!r} ref={y[tuple(idx)]!r}")
    return "\n".join(lines)
