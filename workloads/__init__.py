"""Seeded synthetic inputs for the Ozaki-I GEMM emulator.

This module only draws random matrices. It holds none of the emulation's
arithmetic (no exponents, no slicing, no products), so both the CPU oracle's
tests and the GPU path's tests and benchmark can use the same bytes.

Every generator takes an explicit seed and uses numpy's PCG64 stream
(``numpy.random.default_rng``). Matrices are returned as the mathematical
operands op(A) (m x k) and op(B) (k x n) in plain numpy arrays; callers choose
the memory layout they hand to a BLAS-shaped interface.

The families follow the workloads the paper's application exercises: FP64 GEMM
inside the LU-based inversion of the KKR multiple-scattering matrix, which is
complex and block structured (Section 3.2, Experiments with MuST). The paper's
own inputs (the FeNi3 benchmark of MuST) are not available; these generators
stand in for their shape family only.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_binade",
    "kkr_operands",
    "scaled_gaussian",
    "illcond_operands",
    "batched_problems",
    "complex_normal",
]


def complex_normal(rng: np.random.Generator, shape, scale: float = 1.0) -> np.ndarray:
    """Circular complex Gaussian with E|z|^2 = scale^2."""
    s = scale / np.sqrt(2.0)
    return (rng.standard_normal(shape) * s + 1j * rng.standard_normal(shape) * s).astype(np.complex128)


def uniform_binade(m: int, n: int, k: int, seed: int, emin: int = -4, emax: int = 4,
                   complex_: bool = False):
    """Real (or complex) operands with entries u * 2^e.

    u ~ U(-1, 1) and e ~ uniform integer in [emin, emax], drawn independently for
    every entry (and for the real and imaginary parts separately when complex).
    Returns (A, B) with A of shape (m, k) and B of shape (k, n).
    """
    rng = np.random.default_rng(seed)

    def draw(shape):
        u = rng.uniform(-1.0, 1.0, size=shape)
        e = rng.integers(emin, emax + 1, size=shape)
        return np.ldexp(u, e)

    if complex_:
        A = draw((m, k)) + 1j * draw((m, k))
        B = draw((k, n)) + 1j * draw((k, n))
    else:
        A = draw((m, k))
        B = draw((k, n))
    return A, B


def kkr_operands(nblocks: int, seed: int, block: int = 32, n_rhs: int | None = None):
    """KKR-shaped complex operands A = I - T G and a Gaussian B.

    T is block diagonal with ``block`` x ``block`` complex blocks whose entries
    have magnitude 10^U[-3, 0] (log-uniform in [1e-3, 1]) and a uniform phase.
    G is dense complex Gaussian whose (I, J) block is scaled by 1 / (1 + |I - J|)
    in block distance. A is formed once here in FP64 (it is input data, handed
    to every consumer as bytes). B is complex Gaussian with unit variance and
    ``n_rhs`` columns (default: square).
    """
    rng = np.random.default_rng(seed)
    n = nblocks * block
    n_rhs = n if n_rhs is None else n_rhs
    mag = 10.0 ** rng.uniform(-3.0, 0.0, size=(nblocks, block, block))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(nblocks, block, block))
    T = mag * np.exp(1j * phase)
    G = complex_normal(rng, (n, n))
    bi = np.arange(n) // block
    G = G / (1.0 + np.abs(bi[:, None] - bi[None, :]))
    A = np.eye(n, dtype=np.complex128)
    for I in range(nblocks):
        rows = slice(I * block, (I + 1) * block)
        A[rows, :] -= T[I] @ G[rows, :]
    B = complex_normal(rng, (n, n_rhs))
    return A, B


def scaled_gaussian(m: int, n: int, k: int, seed: int, rmax: int = 30, complex_: bool = True):
    """Gaussian operands with rows of A and columns of B scaled by 2^r.

    r ~ uniform integer in [-rmax, rmax], one per row of A and one per column of
    B. Integer r keeps the scaling exact in FP64.
    """
    rng = np.random.default_rng(seed)
    if complex_:
        A = complex_normal(rng, (m, k))
        B = complex_normal(rng, (k, n))
    else:
        A = rng.standard_normal((m, k))
        B = rng.standard_normal((k, n))
    ra = rng.integers(-rmax, rmax + 1, size=m)
    rb = rng.integers(-rmax, rmax + 1, size=n)
    A = A * np.ldexp(1.0, ra)[:, None]
    B = B * np.ldexp(1.0, rb)[None, :]
    return A, B


def _blocked_complex_normal(seq: np.random.SeedSequence, rows: int, cols: int,
                            nblocks: int) -> np.ndarray:
    """rows x cols circular complex Gaussian (E|z|^2 = 1), drawn in `nblocks`
    row blocks, each from its own child stream of `seq` (so the bytes do not
    depend on how many threads draw them). Real and imaginary parts are
    interleaved draws of one standard normal stream per block."""
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty((rows, cols, 2), dtype=np.float64)
    bounds = np.linspace(0, rows, nblocks + 1).astype(np.int64)
    children = seq.spawn(nblocks)

    def fill(b):
        r0, r1 = int(bounds[b]), int(bounds[b + 1])
        if r1 > r0:
            g = np.random.default_rng(children[b])
            g.standard_normal(out=out[r0:r1])
            out[r0:r1] *= np.sqrt(0.5)

    with ThreadPoolExecutor(max_workers=min(nblocks, 16)) as ex:
        list(ex.map(fill, range(nblocks)))
    return out.view(np.complex128).reshape(rows, cols)


def illcond_operands(m: int, n: int, k: int, seed: int, rmax: int = 30, nblocks: int = 64):
    """Large ill-conditioned complex operands: complex Gaussian A (m x k) and
    B (k x n) with every row of A and every column of B scaled by 2^r,
    r ~ uniform integer in [-rmax, rmax] (exact in FP64).

    The same family as ``scaled_gaussian``, drawn block-parallel so that the
    16384^3 case takes seconds: child streams of SeedSequence(seed) give A's
    row blocks, B's row blocks and the exponents r, in that order.
    """
    seq = np.random.SeedSequence(seed)
    sa, sb, sr = seq.spawn(3)
    A = _blocked_complex_normal(sa, m, k, nblocks)
    B = _blocked_complex_normal(sb, k, n, nblocks)
    g = np.random.default_rng(sr)
    ra = g.integers(-rmax, rmax + 1, size=m)
    rb = g.integers(-rmax, rmax + 1, size=n)
    A *= np.ldexp(1.0, ra)[:, None]
    B *= np.ldexp(1.0, rb)[None, :]
    return A, B


def _spread_matrix(rng, rows, cols, sigma, row_axis):
    """Complex Gaussian entries times 2^(-floor(sigma*u)) with u ~ U[0,1) per
    entry, times 2^r per row (row_axis=0) or column (row_axis=1) with
    r ~ uniform integer in [0, floor(sigma)]."""
    X = complex_normal(rng, (rows, cols))
    off = -np.floor(sigma * rng.uniform(0.0, 1.0, size=(rows, cols))).astype(np.int64)
    X = X * np.ldexp(1.0, off)
    nr = rows if row_axis == 0 else cols
    r = rng.integers(0, int(np.floor(sigma)) + 1, size=nr)
    if row_axis == 0:
        X = X * np.ldexp(1.0, r)[:, None]
    else:
        X = X * np.ldexp(1.0, r)[None, :]
    return X


def batched_sizes(count: int, seed: int, unit: int = 32, jmax: int = 32):
    """m, n, k per problem, each 32*j with P(j) proportional to 1/j (log-uniform
    over multiples of 32 in [32, 1024])."""
    rng = np.random.default_rng(seed)
    j = np.arange(1, jmax + 1)
    p = (1.0 / j) / np.sum(1.0 / j)
    dims = rng.choice(j, size=(count, 3), p=p) * unit
    return dims[:, 0].astype(np.int64), dims[:, 1].astype(np.int64), dims[:, 2].astype(np.int64)


def batched_problems(count: int, seed: int, max_spread: float = 20.0, unit: int = 32,
                     jmax: int = 32, sizes=None):
    """Independent complex problems of uneven size for a batched ZGEMM.

    Sizes follow ``batched_sizes`` unless given as (m, n, k) arrays. Each
    matrix draws its own exponent spread sigma ~ U[0, max_spread] binades:
    entry exponents are offset by -floor(sigma*u), u ~ U[0,1), and each row of
    A (column of B) is scaled by 2^r, r ~ uniform integer in [0, sigma].
    Returns a list of (A, B) pairs and the (m, n, k) arrays.
    """
    if sizes is None:
        ms, ns, ks = batched_sizes(count, seed, unit, jmax)
    else:
        ms, ns, ks = (np.asarray(x, dtype=np.int64) for x in sizes)
    rng = np.random.default_rng(seed + 7919)
    probs = []
    for b in range(count):
        sa, sb = rng.uniform(0.0, max_spread, size=2)
        A = _spread_matrix(rng, int(ms[b]), int(ks[b]), sa, row_axis=0)
        B = _spread_matrix(rng, int(ks[b]), int(ns[b]), sb, row_axis=1)
        probs.append((A, B))
    return probs, (ms, ns, ks)
