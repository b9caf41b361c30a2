"""CPU oracle for splitting p_n and q_{l,n} (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` import this package.  The product library never does, and the two
share no code.

* :mod:`oracle.counts` -- exact integer counts of the paper (Thm countingHyp,
  eq. MisCount, Thm fact_mis) in plain Python integers.
* :mod:`oracle.exact` -- exact integer coefficients of p_n / q_{l,n} and their
  roots by library routines (numpy companion eigenvalues, mpmath polyroots) for
  small degrees; these pin the C oracle from outside.
* this module -- ctypes binding of ``liboracle.so`` (``oracle/oracle.c``): the
  level-line + Newton method in long double / double-double and the
  disk-arithmetic certificate.
"""
import ctypes
import os

import numpy as np

from . import counts  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# statistics slots of oracle.c
STAT_NAMES = [
    "starts", "converged", "diverged", "timeout", "unique", "real", "phase_fail",
    "walk_steps", "lift_steps", "desc_steps", "lookup_mismatch", "discard_hyp",
    "discard_lower", "status", "_14", "_15",
]


def lib():
    """Load liboracle.so, building it first if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build import build
        build()
    L = ctypes.CDLL(_LIB_PATH)
    ld_p = ctypes.POINTER(ctypes.c_longdouble)
    d_p = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    i64_p = ctypes.POINTER(ctypes.c_int64)
    i32_p = ctypes.POINTER(ctypes.c_int32)
    u8_p = ctypes.POINTER(ctypes.c_uint8)
    L.oracle_eval.argtypes = [ctypes.c_int, ctypes.c_int, ld_p, ld_p]
    L.oracle_eval.restype = None
    L.oracle_endpoints.argtypes = [ctypes.c_int, ctypes.c_int, ld_p, ld_p]
    L.oracle_endpoints.restype = None
    L.oracle_starts.argtypes = [ctypes.c_int, ctypes.c_int, i64, ld_p, ld_p, i64_p]
    L.oracle_starts.restype = i64
    L.oracle_split.argtypes = [ctypes.c_int, ctypes.c_int, i64, d_p, d_p, d_p, d_p, i32_p, i64_p]
    L.oracle_split.restype = i64
    L.oracle_split_simple.argtypes = [ctypes.c_int, ctypes.c_int, i64, d_p, d_p, d_p, d_p, i32_p, i64_p]
    L.oracle_split_simple.restype = i64
    L.oracle_certify.argtypes = [ctypes.c_int, ctypes.c_int, i64, d_p, d_p, d_p, d_p, i32_p, u8_p, d_p]
    L.oracle_certify.restype = None
    L.oracle_basin_check.argtypes = [ctypes.c_int, ctypes.c_int, i64, d_p, d_p, d_p, d_p, u8_p]
    L.oracle_basin_check.restype = None
    L.oracle_check_set.argtypes = [i64, d_p, d_p, d_p, i64_p, d_p]
    L.oracle_check_set.restype = None
    L.oracle_check_set_dd.argtypes = [i64, d_p, d_p, d_p, d_p, d_p, i64_p, d_p]
    L.oracle_check_set_dd.restype = None
    L.oracle_disk_enclosure.argtypes = [ctypes.c_int, ctypes.c_int, ld_p, ld_p]
    L.oracle_disk_enclosure.restype = None
    L.oracle_max_threads.argtypes = []
    L.oracle_max_threads.restype = ctypes.c_int
    _lib = L
    return L


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def evaluate(l: int, n: int, c: complex, simple: bool = False):
    """(P(c), P'(c)) for P = q_{l,n} (l = 0: p_n) in long double; with simple,
    P = s_{l,n} = p_{l+n-1} + p_{l-1} (l >= 2)."""
    out = np.zeros(4, dtype=np.longdouble)
    # long doubles travel by pointer: a by-value ctypes c_longdouble goes
    # through a Python float and would lose the extra bits
    if isinstance(c, tuple):
        arg = np.array([c[0], c[1]], dtype=np.longdouble)
    else:
        arg = np.array([c.real, c.imag], dtype=np.longdouble)
    lib().oracle_eval(-(l - 1) if simple else l, n, _ptr(arg, ctypes.c_longdouble), _ptr(out, ctypes.c_longdouble))
    return out


def endpoints(l: int, n: int):
    """Real end points (x_left, x_right) of the level curve |P| = lambda_0."""
    xl = ctypes.c_longdouble()
    xr = ctypes.c_longdouble()
    lib().oracle_endpoints(l, n, ctypes.byref(xl), ctypes.byref(xr))
    return np.longdouble(xl.value), np.longdouble(xr.value)


def starts(l: int, n: int):
    """The 2D+1 level-line starting points of the closed upper half plane
    (start k has P = lambda_0 * i^k), as long-double (re, im) arrays."""
    D = 1 << (l + n - 1)
    ns = 2 * D + 1
    re = np.zeros(ns, dtype=np.longdouble)
    im = np.zeros(ns, dtype=np.longdouble)
    st = np.zeros(16, dtype=np.int64)
    r = lib().oracle_starts(l, n, ns, _ptr(re, ctypes.c_longdouble), _ptr(im, ctypes.c_longdouble),
                            _ptr(st, ctypes.c_int64))
    if r < 0:
        raise RuntimeError(f"oracle_starts({l},{n}) failed with status {r}")
    return re, im, dict(zip(STAT_NAMES, st.tolist()))


class Roots:
    """Roots in the closed upper half plane as double-double (hi + lo)."""

    def __init__(self, re_hi, re_lo, im_hi, im_lo, period, stats):
        self.re_hi, self.re_lo, self.im_hi, self.im_lo = re_hi, re_lo, im_hi, im_lo
        self.period = period
        self.stats = stats

    def __len__(self):
        return len(self.re_hi)

    @property
    def z(self):
        return self.re_hi + 1j * self.im_hi

    def ld(self):
        re = self.re_hi.astype(np.longdouble) + self.re_lo.astype(np.longdouble)
        im = self.im_hi.astype(np.longdouble) + self.im_lo.astype(np.longdouble)
        return re, im


def split(l: int, n: int, simple: bool = False) -> Roots:
    """Split q_{l,n} (l = 0: p_n) with the oracle.  For p_n all 2^(n-1) roots
    are returned with their exact period; for q_{l,n} only Mis(l,n).  With
    simple (l >= 2), Mis(l,n) is found from the roots of the simplified
    polynomial s_{l,n} = p_{l+n-1} + p_{l-1} (eq. polySimple) instead."""
    D = 1 << (l + n - 1)
    cap = D + 1
    a = np.zeros((4, cap), dtype=np.float64)
    per = np.zeros(cap, dtype=np.int32)
    st = np.zeros(16, dtype=np.int64)
    fn = lib().oracle_split_simple if simple else lib().oracle_split
    r = fn(l, n, cap, _ptr(a[0], ctypes.c_double), _ptr(a[1], ctypes.c_double),
           _ptr(a[2], ctypes.c_double), _ptr(a[3], ctypes.c_double),
           _ptr(per, ctypes.c_int32), _ptr(st, ctypes.c_int64))
    stats = dict(zip(STAT_NAMES, st.tolist()))
    if r < 0:
        raise RuntimeError(f"oracle_split({l},{n}, simple={simple}) failed with status {r}: {stats}")
    return Roots(a[0, :r].copy(), a[1, :r].copy(), a[2, :r].copy(), a[3, :r].copy(), per[:r].copy(), stats)


def certify(l: int, n: int, re_hi, im_hi, re_lo=None, im_lo=None, label=None):
    """Disk-arithmetic certificate (Thm proofRoots) of each candidate.

    Returns (flags, radius): flags bit 0 = a unique root of P lies in
    D(candidate, radius); bit 1 = its label (period, or type (l,n)) is proven on
    that disk."""
    re_hi = np.ascontiguousarray(re_hi, dtype=np.float64)
    im_hi = np.ascontiguousarray(im_hi, dtype=np.float64)
    m = len(re_hi)
    re_lo = np.zeros(m) if re_lo is None else np.ascontiguousarray(re_lo, dtype=np.float64)
    im_lo = np.zeros(m) if im_lo is None else np.ascontiguousarray(im_lo, dtype=np.float64)
    if label is None:
        label = np.full(m, n, dtype=np.int32)
    label = np.ascontiguousarray(label, dtype=np.int32)
    ok = np.zeros(m, dtype=np.uint8)
    rad = np.zeros(m, dtype=np.float64)
    lib().oracle_certify(l, n, m, _ptr(re_hi, ctypes.c_double), _ptr(re_lo, ctypes.c_double),
                         _ptr(im_hi, ctypes.c_double), _ptr(im_lo, ctypes.c_double),
                         _ptr(label, ctypes.c_int32), _ptr(ok, ctypes.c_uint8), _ptr(rad, ctypes.c_double))
    return ok, rad


def basin_check(l: int, n: int, re, im, eta, eps):
    """Thm proofContract for each claim: a root lies in D(c, eta), and
    D(c, eps) lies in its Newton basin (c = re + i im as doubles).  Returns a
    bool array: True when the long-double disk-arithmetic check passes."""
    re = np.ascontiguousarray(re, dtype=np.float64)
    im = np.ascontiguousarray(im, dtype=np.float64)
    m = len(re)
    eta = np.ascontiguousarray(np.broadcast_to(eta, (m,)), dtype=np.float64)
    eps = np.ascontiguousarray(np.broadcast_to(eps, (m,)), dtype=np.float64)
    ok = np.zeros(m, dtype=np.uint8)
    lib().oracle_basin_check(l, n, m, _ptr(re, ctypes.c_double), _ptr(im, ctypes.c_double),
                             _ptr(eta, ctypes.c_double), _ptr(eps, ctypes.c_double), _ptr(ok, ctypes.c_uint8))
    return ok.astype(bool)


def disk_enclosure(l: int, n: int, c, R):
    """Disk-arithmetic enclosures at centre c (long double pair or complex):
    returns dict(P, eP, dP, sigma, rho): P(c) in D(P, eP); P'(D(c,R)) in
    D(dP, sigma); P(D(c,R)) in D(P, rho)."""
    re, im = (c if isinstance(c, tuple) else (c.real, c.imag))
    out = np.zeros(7, dtype=np.longdouble)
    arg = np.array([re, im, R], dtype=np.longdouble)
    lib().oracle_disk_enclosure(l, n, _ptr(arg, ctypes.c_longdouble), _ptr(out, ctypes.c_longdouble))
    return dict(P=(out[0], out[1]), eP=out[2], dP=(out[3], out[4]), sigma=out[5], rho=out[6])


def check_set(re, im, radius, re_lo=None, im_lo=None):
    """Global part of Thm certif on a list of certified roots (closed upper
    half plane): returns dict(disjoint, quarter, n_real, n_complex, min_sep).
    With re_lo / im_lo a root is the double-double value re + re_lo,
    im + im_lo (compared in long double).  The list is sorted here by real
    part (the scan needs only that order)."""
    re = np.ascontiguousarray(re, dtype=np.float64)
    im = np.ascontiguousarray(im, dtype=np.float64)
    radius = np.ascontiguousarray(radius, dtype=np.float64)
    out = np.zeros(4, dtype=np.int64)
    ms = ctypes.c_double()
    if re_lo is None and im_lo is None:
        order = np.lexsort((im, re))
        re, im, radius = re[order], im[order], radius[order]
        lib().oracle_check_set(len(re), _ptr(re, ctypes.c_double), _ptr(im, ctypes.c_double),
                               _ptr(radius, ctypes.c_double), _ptr(out, ctypes.c_int64), ctypes.byref(ms))
    else:
        rl = np.zeros_like(re) if re_lo is None else np.ascontiguousarray(re_lo, dtype=np.float64)
        il = np.zeros_like(im) if im_lo is None else np.ascontiguousarray(im_lo, dtype=np.float64)
        # (hi, lo) order is the order of hi + lo for canonical double-doubles
        order = np.lexsort((rl, re))
        re, im, radius, rl, il = re[order], im[order], radius[order], rl[order], il[order]
        lib().oracle_check_set_dd(len(re), _ptr(re, ctypes.c_double), _ptr(rl, ctypes.c_double),
                                  _ptr(im, ctypes.c_double), _ptr(il, ctypes.c_double),
                                  _ptr(radius, ctypes.c_double), _ptr(out, ctypes.c_int64), ctypes.byref(ms))
    return dict(disjoint=bool(out[0]), quarter=bool(out[1]), n_real=int(out[2]),
                n_complex=int(out[3]), min_sep=ms.value)
