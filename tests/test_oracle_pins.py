"""Pins of the CPU oracle against facts fixed outside it.

Each check would fail for a plausible mistake in the oracle: a dropped or
mis-signed term in the orbit recurrence (closed forms at c = -2 and c = 0), a
wrong descent or walk (roots vs mpmath / companion eigenvalues, counts, Vieta),
a wrong period label (Moebius-inverted class sums and per-period counts), a
wrong identification radius (counts, leftmost separation), and a wrong disk
arithmetic radius (containment against 60-digit evaluation, planted mistakes).
"""
import json
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
from oracle import counts, exact

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def all_roots(r):
    """All roots (conjugates added) from an upper-half list, as complex128."""
    z = r.re_hi + 1j * r.im_hi
    return np.concatenate([z, np.conj(z[r.im_hi > 0])])


def total_count(r):
    return int((r.im_hi == 0).sum()) + 2 * int((r.im_hi > 0).sum())


def match_sets(a, b, tol):
    """Nearest-neighbour bijection of two complex point sets within tol."""
    a = np.asarray(a)
    b = np.asarray(b)
    assert len(a) == len(b)
    d = np.abs(a[:, None] - b[None, :])
    ia = d.argmin(axis=1)
    assert len(set(ia.tolist())) == len(a), "not a bijection"
    return float(d[np.arange(len(a)), ia].max())


# --------------------------------------------------------------------- orbit
@pytest.mark.parametrize("n", list(range(2, 32)))
def test_orbit_at_minus_two(n):
    # p_n(-2) = 2 and p_n'(-2) = -(4^n + 2)/6: exact in long double up to n = 31
    P = oracle.evaluate(0, n, (np.longdouble(-2), np.longdouble(0)))
    assert P[0] == 2 and P[1] == 0
    assert P[2] == np.longdouble(-((4 ** n + 2) // 6)) and P[3] == 0


@pytest.mark.parametrize("n", [1, 2, 5, 17, 30])
def test_orbit_at_zero(n):
    P = oracle.evaluate(0, n, (np.longdouble(0), np.longdouble(0)))
    assert P[0] == 0 and P[1] == 0 and P[2] == 1 and P[3] == 0


def test_orbit_matches_exact_coefficients():
    # q_{l,n}(c) and q'(c) at a rational point against exact integer polynomials
    c = Fraction(-3, 4) + 0  # real point; complex point below
    for (l, n) in [(0, 5), (2, 3), (3, 2)]:
        co = exact.q(l, n) if l else exact.p(n)
        val = sum(Fraction(a) * c ** i for i, a in enumerate(co))
        der = sum(i * Fraction(a) * c ** (i - 1) for i, a in enumerate(co) if i)
        P = oracle.evaluate(l, n, (np.longdouble(-0.75), np.longdouble(0)))
        assert abs(float(P[0]) - float(val)) <= 1e-15 * max(1, abs(float(val)))
        assert abs(float(P[2]) - float(der)) <= 1e-15 * max(1, abs(float(der)))
    zc = mpmath.mpc("0.3", "0.55")
    for (l, n) in [(0, 6), (2, 4)]:
        co = exact.q(l, n) if l else exact.p(n)
        with mpmath.workdps(50):
            w = mpmath.mpc(float(zc.real), float(zc.imag))
            val = exact.polyval_mp(co, w)
            der = exact.polyval_mp([i * a for i, a in enumerate(co)][1:], w)
        P = oracle.evaluate(l, n, complex(float(zc.real), float(zc.imag)))
        assert abs(complex(float(P[0]), float(P[1])) - complex(val)) <= 1e-15 * max(1, abs(complex(val)))
        assert abs(complex(float(P[2]), float(P[3])) - complex(der)) <= 1e-15 * max(1, abs(complex(der)))


# --------------------------------------------------------------- small roots
def test_closed_forms_n_le_3():
    hs = GOLD["hyp_small"]
    r1 = oracle.split(0, 1)
    assert len(r1) == 1 and r1.re_hi[0] == hs["Hyp(1)"][0][0] and r1.im_hi[0] == 0
    r2 = oracle.split(0, 2)
    assert sorted(r2.re_hi.tolist()) == [-1.0, 0.0] and np.all(r2.im_hi == 0)
    assert r2.period[r2.re_hi == -1.0][0] == 2 and r2.period[r2.re_hi == 0.0][0] == 1
    # p_3 = z (z^3 + 2 z^2 + z + 1)
    cub = np.roots(GOLD["p3_factor"]["coefficients_high_to_low"])
    ref = np.concatenate([[0.0], cub])
    r3 = oracle.split(0, 3)
    assert total_count(r3) == 4
    assert match_sets(all_roots(r3), ref, 1e-13) < 1e-13


@pytest.mark.parametrize("n", [4, 5, 6])
def test_roots_vs_mpmath_polyroots(n):
    ref = exact.roots_mpmath(exact.p(n), dps=40)
    r = oracle.split(0, n)
    assert total_count(r) == 2 ** (n - 1)
    got = all_roots(r)
    refc = np.array([complex(x) for x in ref])
    assert match_sets(got, refc, 1e-12) < 1e-12
    # double-double accuracy of the oracle against 40 digits
    with mpmath.workdps(40):
        for i in range(len(r)):
            z = mpmath.mpc(mpmath.mpf(r.re_hi[i]) + mpmath.mpf(r.re_lo[i]),
                           mpmath.mpf(r.im_hi[i]) + mpmath.mpf(r.im_lo[i]))
            err = min(abs(z - x) for x in ref)
            assert err < 1e-26, (i, err)


@pytest.mark.parametrize("n", [4, 6])
def test_period_labels_vs_gleason_factors(n):
    # roots labelled k must be exactly the roots of h_k (eq. HypFactor)
    r = oracle.split(0, n)
    for k in counts.divisors(n):
        refk = np.array([complex(x) for x in exact.roots_mpmath(exact.h(k), dps=40)])
        mine = r.re_hi[r.period == k] + 1j * r.im_hi[r.period == k]
        mine = np.concatenate([mine, np.conj(mine[mine.imag > 0])])
        assert match_sets(mine, refk, 1e-12) < 1e-12


@pytest.mark.parametrize("n,tol", [(4, 1e-12), (5, 1e-10), (6, 1e-5)])
def test_companion_eigenvalues(n, tol):
    # float64 eigenvalues of the companion matrix of the exact coefficients;
    # their accuracy degrades with the coefficient growth (worst near -2), but
    # the roots of p_6 are > 1e-3 apart so the bijection is still decisive
    ref = exact.roots_companion(exact.p(n))
    r = oracle.split(0, n)
    assert match_sets(all_roots(r), ref, tol) < tol


# ------------------------------------------------------------------- counts
@pytest.mark.parametrize("n", list(range(1, 17)))
def test_counts_and_period_classes(n):
    r = oracle.split(0, n)
    assert total_count(r) == 2 ** (n - 1)
    assert r.stats["lookup_mismatch"] == 0
    for k in counts.divisors(n):
        sel = r.period == k
        cnt = int((r.im_hi[sel] == 0).sum()) + 2 * int((r.im_hi[sel] > 0).sum())
        assert cnt == counts.hyp_count(k), (n, k)


def top_coefficients(n):
    """(a_{d-1}, a_{d-2}) of p_n from the exact square recurrence on the top
    three coefficients (no root finding involved)."""
    if n <= 4:
        co = exact.p(n)
        d = len(co) - 1
        return co[d - 1], co[d - 2] if d >= 2 else 0
    a, b = top_coefficients(4)
    for _ in range(4, n):
        # (c^D + a c^{D-1} + b c^{D-2} + ...)^2 + c, with 2D - 2 > 1
        a, b = 2 * a, a * a + 2 * b
    return a, b


@pytest.mark.parametrize("n", [2, 3, 5, 8, 11, 14, 16, 18])
def test_vieta_power_sums(n):
    # s1 = -a_{d-1}, s2 = a_{d-1}^2 - 2 a_{d-2}  (Newton's identities)
    a, b = top_coefficients(n)
    s1_exact, s2_exact = -a, a * a - 2 * b
    r = oracle.split(0, n)
    re = r.re_hi.astype(np.longdouble) + r.re_lo
    im = r.im_hi.astype(np.longdouble) + r.im_lo
    w = np.where(r.im_hi > 0, 2, 1).astype(np.longdouble)
    s1 = math.fsum((w * re).astype(np.float64)) + math.fsum(((w * re) - (w * re).astype(np.float64)).astype(np.float64))
    s2 = math.fsum((w * (re * re - im * im)).astype(np.float64))
    assert abs(s1 - s1_exact) <= 1e-9 * max(1, abs(s1_exact))
    assert abs(s2 - s2_exact) <= 1e-9 * max(1, abs(s2_exact))
    if n >= 2:
        assert s1_exact == -(2 ** (n - 2))


@pytest.mark.parametrize("n", [4, 6, 8, 9, 10, 12])
def test_moebius_class_sums(n):
    # sum over Hyp(n) of r = sum_{k|n} mu(n/k) S(k), S(k) = sum of all roots of p_k
    def S(k):
        return 0 if k == 1 else -(2 ** (k - 2))
    expect = sum(counts.mobius(n // k) * S(k) for k in counts.divisors(n))
    r = oracle.split(0, n)
    sel = r.period == n
    got = math.fsum((np.where(r.im_hi[sel] > 0, 2.0, 1.0) * r.re_hi[sel]).tolist())
    assert abs(got - expect) < 1e-9 * max(1, abs(expect))


@pytest.mark.parametrize("n", [9, 10, 12, 14, 16, 18])
def test_leftmost_separation_law(n):
    g = GOLD["leftmost_separation_constant"]
    r = oracle.split(0, n)
    sel = (r.period == n) & (r.im_hi == 0)
    x = np.sort(r.re_hi[sel].astype(np.longdouble) + r.re_lo[sel])
    sep = float(x[1] - x[0])
    assert abs(sep * 4.0 ** n / g["value"] - 1) < g["rel_tol"] + 0.0005
    # and it is the least distance within Hyp(n)
    hyp = r.period == n
    cs = oracle.check_set(r.re_hi[hyp], r.im_hi[hyp], np.zeros(int(hyp.sum())))
    assert abs(cs["min_sep"] - sep) <= 1e-3 * sep


def test_real_root_fraction():
    g = GOLD["real_root_fraction"]
    r = oracle.split(0, 18)
    frac = int((r.im_hi == 0).sum()) / 2 ** 17
    assert g["low"] - 0.01 <= frac <= g["high"] + 0.01


# --------------------------------------------------------------- start set
@pytest.mark.parametrize("ln", [(0, 5), (0, 10), (0, 17), (2, 3)])
def test_start_set(ln):
    l, n = ln
    re, im, st = oracle.starts(l, n)
    D = 2 ** (l + n - 1)
    level = 5 if l == 0 else 100
    assert len(re) == 2 * D + 1 and st["phase_fail"] == 0
    assert np.all(im >= 0)
    assert im[0] == 0 and im[-1] == 0 and re[0] > 0 and re[-1] < -2 + 1e-12
    for k in range(0, 2 * D + 1, max(1, (2 * D + 1) // 64)):
        P = oracle.evaluate(l, n, (re[k], im[k]))
        val = complex(float(P[0]), float(P[1]))
        # rounding noise of the long-double evaluation is about u |P'| |z|
        noise = 64 * 2.0 ** -64 * (abs(complex(float(P[2]), float(P[3]))) * 3 + level)
        assert abs(val - level * [1, 1j, -1, -1j][k % 4]) < noise, k
    z = (re.astype(np.float64) + 1j * im.astype(np.float64))
    zs = np.sort_complex(z)
    assert np.all(np.abs(np.diff(zs)) > 0)


@pytest.mark.parametrize("n", [5, 10, 20])
def test_endpoints_vs_mpmath(n):
    xl, xr = oracle.endpoints(0, n)

    def f(x):
        z = mpmath.mpf(0)
        for _ in range(n):
            z = z * z + x
        return z - 5
    def bisect(a, b):
        fa = f(a)
        for _ in range(160):
            m = (a + b) / 2
            if (f(m) > 0) == (fa > 0):
                a, fa = m, f(m)
            else:
                b = m
        return (a + b) / 2
    with mpmath.workdps(60):
        ref_r = bisect(mpmath.mpf("0.25"), mpmath.mpf(5))
        ref_l = bisect(mpmath.mpf(-3), mpmath.mpf(-2))
    assert abs(float(xr) - float(ref_r)) < 1e-15
    assert abs(float(xl) - float(ref_l)) < 1e-15


# ------------------------------------------------------------ certificate
@pytest.mark.parametrize("n", [6, 12])
def test_certificate_accepts_oracle_roots(n):
    r = oracle.split(0, n)
    ok, rad = oracle.certify(0, n, r.re_hi, r.im_hi, r.re_lo, r.im_lo, r.period)
    assert np.all(ok == 3)
    assert rad.max() < 1e-15
    cs = oracle.check_set(r.re_hi, r.im_hi, rad)
    assert cs["disjoint"] and cs["quarter"]
    assert cs["n_real"] + 2 * cs["n_complex"] == 2 ** (n - 1)


def test_certificate_rejects_planted_mistakes():
    n = 10
    r = oracle.split(0, n)
    re, im = r.re_hi.copy(), r.im_hi.copy()
    # a root moved by 1e-3 is no longer certified within a small radius
    re[17] += 1e-3
    ok, rad = oracle.certify(0, n, re, im, label=r.period)
    assert not (ok[17] & 1 and rad[17] <= 1e-10)
    # a wrong period label fails the label bit only
    lab = r.period.copy()
    i = int(np.where(lab == n)[0][0])
    lab[i] = 5
    ok, rad = oracle.certify(0, n, r.re_hi, r.im_hi, r.re_lo, r.im_lo, lab)
    assert ok[i] & 1 and not ok[i] & 2
    # a duplicated root (replacing another one) breaks disjointness and count
    re, im = r.re_hi.copy(), r.im_hi.copy()
    j = int(np.where(im > 0)[0][3])
    re[j + 1], im[j + 1] = re[j], im[j]
    ok, rad = oracle.certify(0, n, re, im)
    cs = oracle.check_set(re, im, rad)
    assert not cs["disjoint"]
    # a dropped root breaks the count
    keep = np.ones(len(r), bool)
    keep[j] = False
    ok, rad = oracle.certify(0, n, r.re_hi[keep], r.im_hi[keep])
    cs = oracle.check_set(r.re_hi[keep], r.im_hi[keep], rad)
    assert cs["n_real"] + 2 * cs["n_complex"] != 2 ** (n - 1)


def _mp_q(l, n, w):
    """q_{l,n}(w), q'(w) at mpmath precision through the orbit (no coefficient
    cancellation, unlike Horner on the huge exact coefficients near -2)."""
    z = dz = zl = dzl = mpmath.mpc(0)
    for k in range(1, l + n + 1):
        dz = 2 * z * dz + 1
        z = z * z + w
        if k == l:
            zl, dzl = z, dz
    return z - zl, dz - dzl


def _mp(x):
    a, b = x.as_integer_ratio()
    return mpmath.mpf(a) / b


@pytest.mark.parametrize("ln,R", [((0, 8), 1e-12), ((0, 8), 1e-6), ((0, 12), 1e-9), ((2, 4), 1e-8), ((0, 5), 0.05)])
def test_disk_enclosure_contains_exact_values(ln, R):
    """P(c), P(D(c,R)) and P'(D(c,R)) evaluated at 60 digits stay inside the
    disks of Thm diskArithmetic computed by the oracle."""
    l, n = ln
    rng = np.random.default_rng(1234 + n)
    r = oracle.split(0, max(n - 2, 1))
    cs = (r.re_hi + 1j * r.im_hi)[:: max(1, len(r) // 6)][:6]
    cs = np.concatenate([cs, [0.3 + 0.5j, -1.2 + 0.1j]])
    for c in cs:
        cre, cim = np.longdouble(c.real), np.longdouble(c.imag)
        enc = oracle.disk_enclosure(l, n, (cre, cim), R)
        with mpmath.workdps(60):
            cm = mpmath.mpc(_mp(cre), _mp(cim))
            Pc = mpmath.mpc(_mp(enc["P"][0]), _mp(enc["P"][1]))
            dPc = mpmath.mpc(_mp(enc["dP"][0]), _mp(enc["dP"][1]))
            assert abs(_mp_q(l, n, cm)[0] - Pc) <= _mp(enc["eP"])
            for t in range(48):
                rho = R if t < 24 else R * rng.random()
                w = cm + rho * mpmath.expj(2 * mpmath.pi * rng.random())
                Pw, dPw = _mp_q(l, n, w)
                assert abs(Pw - Pc) <= _mp(enc["rho"])
                assert abs(dPw - dPc) <= _mp(enc["sigma"])


# ----------------------------------------------------------- Misiurewicz
def test_mis_small_closed_forms():
    r = oracle.split(2, 1)
    assert len(r) == 1 and r.re_hi[0] == GOLD["mis_small"]["Mis(2,1)"][0][0] and r.im_hi[0] == 0
    r = oracle.split(2, 2)  # s_{2,2} = c (c + 2)(c^2 + 1): Mis(2,2) = {i, -i}
    assert len(r) == 1 and abs(r.re_hi[0]) < 1e-30 and r.im_hi[0] == 1.0
    r = oracle.split(3, 1)  # m_{3,1} = c^3 + 2c^2 + 2c + 2
    ref = np.roots([1, 2, 2, 2])
    assert match_sets(all_roots(r), ref, 1e-13) < 1e-13


@pytest.mark.parametrize("ln", [(2, 3), (2, 4), (3, 2), (3, 3), (4, 2), (2, 5)])
def test_mis_vs_exact_reduced_polynomial(ln):
    l, n = ln
    ref = np.array([complex(x) for x in exact.roots_mpmath(exact.m(l, n), dps=40)])
    r = oracle.split(l, n)
    assert total_count(r) == counts.mis_count(l, n) == len(ref)
    assert match_sets(all_roots(r), ref, 1e-12) < 1e-12


@pytest.mark.parametrize("order", list(range(3, 13)))
def test_mis_counts(order):
    for l in range(2, order):
        n = order - l
        r = oracle.split(l, n)
        assert total_count(r) == counts.mis_count(l, n), (l, n)


@pytest.mark.parametrize("ln", [(13, 1), (14, 2), (15, 1), (20, 2)])
def test_mis_endpoints_large_preperiod(ln):
    """Real end points of |q_{l,n}| = 100 (Section 6.3.1) where the far end of
    the bisection bracket overflows: checked against the orbit in mpmath (no
    overflow there) -- q crosses the level inside a 1e-12 bracket of each."""
    l, n = ln
    xl, xr = oracle.endpoints(l, n)

    def q(x):
        z, zl = mpmath.mpf(0), None
        for k in range(1, l + n + 1):
            z = z * z + x
            if k == l:
                zl = z
        return z - zl - 100

    for x in (xl, xr):
        a, b = mpmath.mpf(float(x)) - mpmath.mpf(1e-12), mpmath.mpf(float(x)) + mpmath.mpf(1e-12)
        assert (q(a) > 0) != (q(b) > 0), (ln, float(x))
    assert 0.25 < float(xr) < 1.0 and float(xl) < -2.0


@pytest.mark.parametrize("ln", [(3, 15), (6, 13), (2, 16), (4, 14)])
def test_mis_counts_order_18_19(ln):
    """Orders where descents settle on the multiple roots of q_{l,n} (the
    centres Hyp(k), k | n, Thm fact_mis) closely enough to pass any fixed
    zero threshold: the count must still be exactly |Mis(l,n)| (eq. MisCount)
    and no returned point may be a centre."""
    l, n = ln
    r = oracle.split(l, n)
    assert total_count(r) == counts.mis_count(l, n), ln
    assert not np.any((r.im_hi > 0) & (r.im_hi < 1e-14))


@pytest.mark.parametrize("ln", [(13, 1), (13, 2), (14, 1), (14, 2), (15, 1)])
def test_mis_counts_large_preperiod(ln):
    l, n = ln
    r = oracle.split(l, n)
    assert total_count(r) == counts.mis_count(l, n), ln


def test_mis_certificates_prove_the_type():
    for (l, n) in [(2, 4), (3, 3), (4, 6)]:
        r = oracle.split(l, n)
        ok, rad = oracle.certify(l, n, r.re_hi, r.im_hi, r.re_lo, r.im_lo)
        assert np.all(ok == 3), (l, n, np.bincount(ok))
        cs = oracle.check_set(r.re_hi, r.im_hi, rad)
        assert cs["disjoint"] and cs["n_real"] + 2 * cs["n_complex"] == counts.mis_count(l, n)


def test_degree_identity_and_q24_factorization():
    # eq. MisDeg on the counting functions
    for l in range(0, 9):
        for n in range(1, 9):
            if l == 1:
                continue
            tot = sum(counts.eta(l, k) * counts.hyp_count(k) + sum(counts.mis_count(j, k) for j in range(2, l + 1))
                      for k in counts.divisors(n)) if l >= 2 else None
            if tot is not None:
                assert tot == 2 ** (l + n - 1), (l, n)
    # the worked example of Appendix A, in exact integer arithmetic
    e = GOLD["q24_factorization"]["exponents"]
    prod = [1]
    for poly, k in [(exact.h(1), e["h1"]), (exact.h(2), e["h2"]), (exact.h(4), e["h4"]),
                    (exact.m(2, 1), e["m21"]), (exact.m(2, 2), e["m22"]), (exact.m(2, 4), e["m24"])]:
        for _ in range(k):
            prod = exact.pmul(prod, list(poly))
    assert prod == list(exact.q(2, 4))
    assert counts.eta(2, 1) == 3 and counts.eta(2, 2) == 2 and counts.eta(2, 4) == 2


# --------------------------------------------------------------- Newton basin
# Thm proofContract, checked by the oracle in long-double disk arithmetic.

def test_basin_check_closed_form_p2():
    """p_2 = c^2 + c, roots 0 and -1, P' = 2c + 1: P'(D(r, eps)) = D(P'(r), 2 eps)
    with |P'(r)| = 1, so the condition |centre| > 5 radius holds exactly for
    eps < 1/10; eps must also exceed 3 eta."""
    ok = oracle.basin_check(0, 2, [0.0, 0.0, -1.0, -1.0], [0.0] * 4, 1e-20, [0.0999, 0.1001, 0.0999, 0.1001])
    assert list(ok) == [True, False, True, False]
    assert not oracle.basin_check(0, 2, [0.0], [0.0], 0.04, [0.0999])[0]  # eps <= 3 eta
    # p_1 = c: P' = 1 everywhere, any eps above 3 eta
    assert oracle.basin_check(0, 1, [0.0], [0.0], 1e-20, [0.25])[0]


def _largest_basin(l, n, z, eta):
    eps = np.zeros(len(z))
    for k in range(2, 60):
        ok = oracle.basin_check(l, n, z.real, z.imag, eta, 2.0 ** -k)
        eps = np.where((eps == 0) & ok, 2.0 ** -k, eps)
    return eps


def _newton_pn(n, c, iters=80):
    for _ in range(iters):
        z = np.zeros_like(c)
        dz = np.zeros_like(c)
        for _k in range(n):
            dz = 2 * z * dz + 1
            z = z * z + c
        c = c - z / dz
    return c


@pytest.mark.parametrize("n", [5, 7])
def test_basin_disks_converge_under_newton(n):
    """Newton's method started anywhere in a disk the check accepts converges
    to that disk's root (sampled points, double precision): the consequence
    Thm proofContract asserts, tested by running the method."""
    r = oracle.split(0, n)
    z = r.re_hi + 1j * r.im_hi
    eps = _largest_basin(0, n, z, 1e-18)
    assert np.all(eps > 0)
    rng = np.random.default_rng(11)
    for zi, ei in zip(z, eps):
        rad = ei * np.sqrt(rng.random(64))
        ang = 2 * np.pi * rng.random(64)
        pts = zi + rad * np.exp(1j * ang)
        end = _newton_pn(n, pts)
        assert np.max(np.abs(end - zi)) < 1e-10, (zi, ei)


@pytest.mark.parametrize("n", [6, 8])
def test_basin_check_rejects_disks_holding_two_roots(n):
    """A disk that reaches another root (or the conjugate) cannot lie in one
    basin: the check must refuse eps = the distance to the nearest other root
    (a check that accepted everything would fail here)."""
    r = oracle.split(0, n)
    z = r.re_hi + 1j * r.im_hi
    allz = np.concatenate([z, np.conj(z[r.im_hi > 0])])
    d = np.abs(z[:, None] - allz[None, :])
    d[d == 0] = np.inf
    near = d.min(axis=1)
    assert not np.any(oracle.basin_check(0, n, z.real, z.imag, 1e-18, near * 1.01))


# ------------------------------------------- simplified polynomials s_{l,n}
# eq. polySimple / eq. polyMisSimple: s_{l,n} = q_{l,n} / q_{l-1,n}
# = p_{l+n-1} + p_{l-1}, with simple roots Hyp(k), k | gcd(n, l-1), and
# Mis(l,k), k | n.

@pytest.mark.parametrize("l,n", [(2, 1), (2, 4), (3, 3), (4, 2), (5, 4), (3, 6)])
def test_simple_polynomial_is_the_exact_quotient(l, n):
    """q_{l,n} = s_{l,n} q_{l-1,n} as integer polynomials, s_{l,n} =
    p_{l+n-1} + p_{l-1}, and s_{l,n} = prod h_k (k | gcd(n, l-1)) prod m_{l,k}
    (k | n), so its degree 2^(l+n-2) splits into those counts."""
    from oracle import exact
    assert exact.pmul(list(exact.s(l, n)), list(exact.q(l - 1, n))) == list(exact.q(l, n))
    deg = len(exact.s(l, n)) - 1
    assert deg == 2 ** (l + n - 2)
    g = math.gcd(n, l - 1)
    total = sum(counts.hyp_count(k) for k in counts.divisors(g)) + sum(
        counts.mis_count(l, k) for k in counts.divisors(n))
    assert total == deg


@pytest.mark.parametrize("l,n", [(2, 3), (3, 2), (4, 4), (3, 6)])
def test_simple_evaluation_matches_exact_polynomial(l, n):
    """The oracle's orbit evaluation of s_{l,n} and its derivative against the
    exact integer coefficients (60 digits) at seeded points."""
    import mpmath
    from oracle import exact
    co = list(exact.s(l, n))
    dco = [k * co[k] for k in range(1, len(co))]
    rng = np.random.default_rng(5)
    for _ in range(12):
        c = complex(rng.uniform(-2, 0.5), rng.uniform(-1.2, 1.2))
        P = oracle.evaluate(l, n, c, simple=True)
        Pe = complex(exact.polyval_mp(co, mpmath.mpc(c)))
        dPe = complex(exact.polyval_mp(dco, mpmath.mpc(c)))
        assert abs(complex(float(P[0]), float(P[1])) - Pe) <= 1e-15 * (1 + abs(Pe))
        assert abs(complex(float(P[2]), float(P[3])) - dPe) <= 1e-15 * (1 + abs(dPe))


@pytest.mark.parametrize("l,n", [(2, 1), (2, 2), (3, 1), (2, 4), (3, 4), (4, 3), (5, 4), (3, 8), (6, 6), (2, 10)])
def test_simple_split_equals_q_split(l, n):
    """Mis(l,n) found from the roots of s_{l,n} (half the degree, simple
    roots, its own level line and starts) equals Mis(l,n) found from
    q_{l,n}: two independent routes to the same set."""
    a = oracle.split(l, n)
    b = oracle.split(l, n, simple=True)
    za = np.sort_complex((a.re_hi + a.re_lo) + 1j * (a.im_hi + a.im_lo))
    zb = np.sort_complex((b.re_hi + b.re_lo) + 1j * (b.im_hi + b.im_lo))
    assert len(za) == len(zb)
    assert np.max(np.abs(za - zb)) < 1e-20


@pytest.mark.parametrize("l,n", [(2, 12), (4, 10), (7, 7), (12, 2), (3, 13)])
def test_simple_split_counts(l, n):
    """|Mis(l,n)| (eq. MisCount) from s_{l,n} at orders 14 to 16."""
    b = oracle.split(l, n, simple=True)
    total = int(np.sum(b.im_hi == 0)) + 2 * int(np.sum(b.im_hi != 0))
    assert total == counts.mis_count(l, n)
