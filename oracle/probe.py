"""Randomized residual probe: the plain CPU definition.

TEST INFRASTRUCTURE ONLY.

For nvec sign vectors x_v with entries +-1 taken from the top bit of
SplitMix64(seed + v*n + j) (Steele, Lea and Flood 2014; the 64-bit finalizer
of Vigna's published splitmix64), the residual r_v = C x_v - op(A)(op(B) x_v)
is computed exactly in rational arithmetic, u = |op(A)| (|op(B)| 1) with
entrywise moduli, and
    est_i = sqrt(mean_v |r_v,i|^2) * sqrt(n) / u_i
(0 when u_i = 0 and r = 0, +inf when u_i = 0 and r != 0). It estimates the
componentwise error scale of row i of C as an approximation of op(A) op(B):
random signs make |r_v,i| about the root-mean-square error of the row times
u_i / sqrt(n).
"""
from __future__ import annotations

import math

import numpy as np

from .exact import exact_dot, exact_dot_q
from .ozaki import op

MASK = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One output of SplitMix64 from state x (the state is advanced by the
    golden-ratio increment first, as in the published generator)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def signs(seed: int, nvec: int, n: int) -> np.ndarray:
    """(nvec, n) array of +-1.0."""
    out = np.empty((nvec, n))
    for v in range(nvec):
        for j in range(n):
            out[v, j] = -1.0 if splitmix64((seed + v * n + j) & MASK) >> 63 else 1.0
    return out


def probe_est(transa, transb, A, B, C, nvec: int, seed: int) -> np.ndarray:
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B) or np.iscomplexobj(C)
    dt = np.complex128 if cplx else np.float64
    opA = op(np.asarray(A, dtype=dt), transa)
    opB = op(np.asarray(B, dtype=dt), transb)
    C = np.asarray(C, dtype=dt)
    m, k = opA.shape
    n = opB.shape[1]
    X = signs(seed, nvec, n)
    ub = np.abs(opB).sum(axis=1) if n else np.zeros(k)
    u = np.abs(opA) @ ub if k else np.zeros(m)
    ss = np.zeros(m)
    for v in range(nvec):
        x = X[v]
        # w = op(B) x exactly (per component)
        wr = [exact_dot(opB.real[l], x) for l in range(k)]
        wi = [exact_dot(opB.imag[l], x) for l in range(k)] if cplx else None
        for i in range(m):
            yr = exact_dot(C.real[i], x)
            if cplx:
                zr = exact_dot_q(list(opA.real[i]) + list(-opA.imag[i]), wr + wi)
                zi = exact_dot_q(list(opA.real[i]) + list(opA.imag[i]), wi + wr)
                yi = exact_dot(C.imag[i], x)
                r2 = (yr - zr) ** 2 + (yi - zi) ** 2
            else:
                zr = exact_dot_q(list(opA[i]), wr)
                r2 = (yr - zr) ** 2
            ss[i] += float(r2)
    est = np.empty(m)
    for i in range(m):
        if u[i] == 0:
            est[i] = 0.0 if ss[i] == 0 else math.inf
        else:
            est[i] = math.sqrt(ss[i] / nvec) * math.sqrt(n) / u[i]
    return est
