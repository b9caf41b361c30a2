"""Pins of the CPU oracle at the sizes where it judges the headline batch.

The GPU parity tests compare p_21 .. p_25 element by element with
``oracle.split``, so the oracle is pinned there too, by facts fixed outside
it: the exact count 2^(n-1) and the per-period counts of eq. HypCount
(Thm countingHyp), Vieta's first two power sums from the exact top
coefficients, the leftmost separation 118.4 / 4^n of Section 6.3.2, and its
own certificate (Thm proofRoots, Thm certif) over every root.

The global set check of the certificate (disjoint disks, and the
quarter-separation reading) is pinned on planted configurations: a pair
closer than four radii must fail the quarter test while its disks stay
disjoint, and double-double roots closer than the FP64 spacing must be told
apart through their low parts.
"""
import functools
import math

import numpy as np
import pytest

import oracle
from oracle import counts, exact

pytestmark = pytest.mark.slow


@functools.lru_cache(maxsize=None)
def split(n):
    return oracle.split(0, n)


def top_coefficients(n):
    """(a_{d-1}, a_{d-2}) of p_n from the exact square recurrence on the top
    coefficients: (c^D + a c^(D-1) + b c^(D-2) + ...)^2 + c."""
    co = exact.p(4)
    d = len(co) - 1
    a, b = co[d - 1], co[d - 2]
    for _ in range(4, n):
        a, b = 2 * a, a * a + 2 * b
    return a, b


@pytest.mark.parametrize("n", [22, 24])
def test_large_split_counts_per_period(n):
    r = split(n)
    assert r.stats["status"] == 0 and r.stats["lookup_mismatch"] == 0
    assert int((r.im_hi == 0).sum()) + 2 * int((r.im_hi > 0).sum()) == 2 ** (n - 1)
    for k in counts.divisors(n):
        sel = r.period == k
        cnt = int((r.im_hi[sel] == 0).sum()) + 2 * int((r.im_hi[sel] > 0).sum())
        assert cnt == counts.hyp_count(k), (n, k, cnt)


@pytest.mark.parametrize("n", [22, 24])
def test_large_split_vieta(n):
    # Newton's identities: s1 = -a_{d-1}, s2 = a_{d-1}^2 - 2 a_{d-2}
    a, b = top_coefficients(n)
    s1_exact, s2_exact = -a, a * a - 2 * b
    assert s1_exact == -(2 ** (n - 2))
    r = split(n)
    re = r.re_hi.astype(np.longdouble) + r.re_lo
    im = r.im_hi.astype(np.longdouble) + r.im_lo
    w = np.where(r.im_hi > 0, 2, 1).astype(np.longdouble)
    s1 = math.fsum((w * re).astype(np.float64).tolist())
    s2 = math.fsum((w * (re * re - im * im)).astype(np.float64).tolist())
    assert abs(s1 - s1_exact) <= 1e-9 * abs(s1_exact), (s1, s1_exact)
    assert abs(s2 - s2_exact) <= 1e-9 * max(1, abs(s2_exact)), (s2, s2_exact)


@pytest.mark.parametrize("n", [22, 24])
def test_large_split_leftmost_separation(n):
    # Section 6.3.2: the two leftmost real centres of period n are 118.4 / 4^n apart
    r = split(n)
    sel = (r.period == n) & (r.im_hi == 0)
    x = np.sort(r.re_hi[sel].astype(np.longdouble) + r.re_lo[sel])
    assert abs(float(x[1] - x[0]) * 4.0 ** n / 118.4 - 1) < 0.002


@pytest.mark.parametrize("n", [22, 24])
def test_large_split_certified_by_oracle(n):
    """Every root in a unique-root disk of radius <= 1e-10 with its period
    proven, the disks disjoint and quarter-separated, and the count equal to
    the degree: by Thm certif the list is the root set of p_n."""
    r = split(n)
    ok, rad = oracle.certify(0, n, r.re_hi, r.im_hi, r.re_lo, r.im_lo, r.period)
    assert np.all(ok == 3)
    assert rad.max() <= 1e-10
    cs = oracle.check_set(r.re_hi, r.im_hi, rad, r.re_lo, r.im_lo)
    assert cs["disjoint"] and cs["quarter"]
    assert cs["n_real"] + 2 * cs["n_complex"] == 2 ** (n - 1)
    # the least distance over all periods lies below the leftmost pair of
    # Hyp(n) (118.4 / 4^n): for even n a centre of period n/2 and its
    # satellite of period n come closer (about 59.2 / 4^n)
    assert 50.0 < cs["min_sep"] * 4.0 ** n < 118.4


def test_check_set_quarter_flag_refuses_a_close_pair():
    """Disks of radius d/3 around the two closest real roots of p_10 (d
    apart) are disjoint (2d/3 < d) but not quarter-separated (d < 4d/3);
    radius 0.51 d makes them overlap.  A non-real root at height y and its
    conjugate (2y apart): radius 0.6 y keeps the disks disjoint but not
    quarter-separated, 1.1 y makes them overlap."""
    r = oracle.split(0, 10)
    ok, rad = oracle.certify(0, 10, r.re_hi, r.im_hi, r.re_lo, r.im_lo, r.period)
    cs = oracle.check_set(r.re_hi, r.im_hi, rad)
    assert cs["disjoint"] and cs["quarter"]
    real = np.where(r.im_hi == 0)[0]
    x = r.re_hi[real]
    o = np.argsort(x)
    gaps = np.diff(x[o])
    m = int(np.argmin(gaps))
    i, j = real[o[m]], real[o[m + 1]]
    dij = gaps[m]
    rad2 = rad.copy()
    rad2[i] = rad2[j] = dij / 3
    cs = oracle.check_set(r.re_hi, r.im_hi, rad2)
    assert cs["disjoint"] and not cs["quarter"]
    rad2[i] = rad2[j] = dij * 0.51
    cs = oracle.check_set(r.re_hi, r.im_hi, rad2)
    assert not cs["disjoint"] and not cs["quarter"]
    # conjugate pair, planted
    re, im = np.array([-1.0, 0.3]), np.array([0.0, 1e-6])
    cs = oracle.check_set(re, im, np.array([1e-12, 0.4e-6]))
    assert cs["disjoint"] and cs["quarter"] and cs["n_real"] == 1 and cs["n_complex"] == 1
    cs = oracle.check_set(re, im, np.array([1e-12, 0.6e-6]))
    assert cs["disjoint"] and not cs["quarter"]
    cs = oracle.check_set(re, im, np.array([1e-12, 1.1e-6]))
    assert not cs["disjoint"]


def test_check_set_double_double_values():
    """Two roots closer than the FP64 spacing (same high parts, low parts
    1e-17 apart, as next to -2 at order 30) are apart in double-double: with
    radii 2e-18 their disks are disjoint and quarter-separated; radii 3e-18
    are disjoint but not quarter-separated; 6e-18 overlap; without the low
    parts the two coincide.  A non-real root 1e-17 above the axis next to
    them: its conjugate disk is 2e-17 away."""
    x = -1.9999999999999998
    re = np.array([-1.5, x, x, 0.25])
    re_lo = np.array([0.0, 0.0, 1e-17, 0.0])
    im = np.zeros(4)
    im_lo = np.zeros(4)
    rad = np.array([1e-12, 2e-18, 2e-18, 1e-12])
    cs = oracle.check_set(re, im, rad, re_lo, im_lo)
    assert cs["disjoint"] and cs["quarter"] and cs["n_real"] == 4
    assert abs(cs["min_sep"] - 1e-17) < 1e-19
    cs = oracle.check_set(re, im, np.array([1e-12, 3e-18, 3e-18, 1e-12]), re_lo, im_lo)
    assert cs["disjoint"] and not cs["quarter"]
    cs = oracle.check_set(re, im, np.array([1e-12, 6e-18, 6e-18, 1e-12]), re_lo, im_lo)
    assert not cs["disjoint"]
    # high parts alone: the pair is one point
    assert not oracle.check_set(re, im, rad)["disjoint"]
    im2 = np.array([0.0, 0.0, 1e-17, 0.0])
    cs = oracle.check_set(re, im2, np.array([1e-12, 1e-19, 3e-18, 1e-12]), re_lo, im_lo)
    assert cs["n_real"] == 3 and cs["n_complex"] == 1
    assert cs["disjoint"] and cs["quarter"]
    cs = oracle.check_set(re, im2, np.array([1e-12, 1e-19, 6e-18, 1e-12]), re_lo, im_lo)
    assert cs["disjoint"] and not cs["quarter"]
