"""Exact integer polynomials of the paper and their roots by library routines.

These pin the C oracle from outside: the coefficients come from exact integer
algebra (Python ints), the roots from numpy's companion-matrix eigenvalues
(Section 3, eigenvalue methods) or mpmath's polyroots, never from the level-line
method.  Polynomials are little-endian coefficient lists.

* p_0 = 0, p_{k+1} = p_k^2 + z                       (eq. def:hyp_poly)
* q_{l,n} = p_{l+n} - p_l                            (eq. def:mis_poly)
* p_n = prod_{k | n} h_k                             (eq. HypFactor)
* s_{l,n} = p_{l+n-1} + p_{l-1}
        = prod_{k | gcd(n,l-1)} h_k * prod_{k | n} m_{l,k}   (eq. polyMisSimple)
"""
from functools import lru_cache
from math import gcd

import numpy as np

from .counts import divisors


def padd(a, b):
    n = max(len(a), len(b))
    return trim([(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)])


def psub(a, b):
    return padd(a, [-x for x in b])


def pmul(a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x:
            for j, y in enumerate(b):
                out[i + j] += x * y
    return trim(out)


def trim(a):
    a = list(a)
    while len(a) > 1 and a[-1] == 0:
        a.pop()
    return a


def pdivexact(a, b):
    """Exact division of integer polynomials (b monic); raises if inexact."""
    a = list(a)
    if b[-1] != 1:
        raise ValueError("divisor must be monic")
    db = len(b) - 1
    q = [0] * max(len(a) - db, 1)
    for i in range(len(a) - 1, db - 1, -1):
        c = a[i]
        if c:
            q[i - db] = c
            for j in range(db + 1):
                a[i - db + j] -= c * b[j]
    if any(a[:db]):
        raise ArithmeticError("division is not exact")
    return trim(q)


@lru_cache(maxsize=None)
def p(n: int):
    a = [0]
    for _ in range(n):
        a = padd(pmul(a, a), [0, 1])
    return tuple(a)


def q(l: int, n: int):
    return tuple(psub(list(p(l + n)), list(p(l))))


@lru_cache(maxsize=None)
def h(n: int):
    """Gleason polynomial h_n (roots: Hyp(n))."""
    a = list(p(n))
    for k in divisors(n)[:-1]:
        a = pdivexact(a, list(h(k)))
    return tuple(a)


def s(l: int, n: int):
    return tuple(padd(list(p(l + n - 1)), list(p(l - 1))))


@lru_cache(maxsize=None)
def m(l: int, n: int):
    """Reduced Misiurewicz polynomial m_{l,n} (roots: Mis(l,n)), l >= 2."""
    a = list(s(l, n))
    for k in divisors(gcd(n, l - 1)):
        a = pdivexact(a, list(h(k)))
    for k in divisors(n)[:-1]:
        a = pdivexact(a, list(m(l, k)))
    return tuple(a)


def roots_companion(coeffs):
    """Roots by eigenvalues of the companion matrix (float64)."""
    c = np.array([float(x) for x in coeffs], dtype=np.float64)
    return np.roots(c[::-1])


def roots_mpmath(coeffs, dps: int = 60):
    """Roots by mpmath.polyroots at dps digits (list of mpc)."""
    import mpmath
    with mpmath.workdps(dps):
        return mpmath.polyroots(list(coeffs)[::-1], maxsteps=400, extraprec=4 * dps)


def upper_half(roots, tol=1e-20):
    """Roots with Im >= 0 (conjugate pairs kept once)."""
    return [r for r in roots if r.imag >= -tol]


def polyval_mp(coeffs, z, dps: int = 60):
    import mpmath
    with mpmath.workdps(dps):
        acc = mpmath.mpc(0)
        for c in reversed(coeffs):
            acc = acc * z + c
        return acc
