"""Exact entries of op(A) op(B) with Python integers and fractions.

TEST INFRASTRUCTURE ONLY. Every FP64 value is a dyadic rational n / 2^d; a dot
product of such values is summed exactly as one big integer over a common power
of two. Used to check the double-double reference and for tiny brute-force
checks of the emulation model.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from .ozaki import op


def _dyadic(x: float):
    """x = num / 2^d with integer num and d >= 0."""
    num, den = float(x).as_integer_ratio()
    d = den.bit_length() - 1
    return num, d


def exact_dot(a, b) -> Fraction:
    """sum_l a_l b_l exactly, for real float sequences."""
    terms = []
    dmax = 0
    for x, y in zip(a, b):
        nx, dx = _dyadic(x)
        ny, dy = _dyadic(y)
        terms.append((nx * ny, dx + dy))
        dmax = max(dmax, dx + dy)
    total = 0
    for num, d in terms:
        total += num << (dmax - d)
    return Fraction(total, 1 << dmax)


def exact_entries(transa, transb, A, B, rows, cols):
    """Exact values of the entries (rows[x], cols[x]) as Fractions. Complex data
    gives (re, im) tuples of Fractions."""
    complex_ = np.iscomplexobj(A) or np.iscomplexobj(B)
    dt = np.complex128 if complex_ else np.float64
    opA = op(np.asarray(A, dtype=dt), transa)
    opB = op(np.asarray(B, dtype=dt), transb)
    out = []
    for i, j in zip(rows, cols):
        a = opA[int(i), :]
        b = opB[:, int(j)]
        if complex_:
            re = exact_dot(np.concatenate([a.real, -a.imag]), np.concatenate([b.real, b.imag]))
            im = exact_dot(np.concatenate([a.real, a.imag]), np.concatenate([b.imag, b.real]))
            out.append((re, im))
        else:
            out.append(exact_dot(a, b))
    return out


def to_float(v) -> float | complex:
    """Round an exact value (Fraction or (re, im)) to the nearest FP64; Python's
    float(Fraction) is correctly rounded."""
    if isinstance(v, tuple):
        return complex(float(v[0]), float(v[1]))
    return float(v)


def _dyadic_q(x):
    """num / 2^d for a float or a Fraction with a power-of-two denominator."""
    if isinstance(x, Fraction):
        num, den = x.numerator, x.denominator
    else:
        num, den = float(x).as_integer_ratio()
    d = den.bit_length() - 1
    if den != 1 << d:
        raise ValueError("not a dyadic rational")
    return num, d


def exact_dot_q(a, b) -> Fraction:
    """sum_l a_l b_l exactly for floats and dyadic Fractions."""
    terms = []
    dmax = 0
    for x, y in zip(a, b):
        nx, dx = _dyadic_q(x)
        ny, dy = _dyadic_q(y)
        terms.append((nx * ny, dx + dy))
        dmax = max(dmax, dx + dy)
    total = 0
    for num, d in terms:
        total += num << (dmax - d)
    return Fraction(total, 1 << dmax)
