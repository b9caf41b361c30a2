"""Exact counts of the paper, in plain Python integers (oracle side).

* |Hyp(n)| = sum_{k | n} mu(n/k) 2^(k-1)            (Thm countingHyp, eq. HypCount)
* |Mis(l,n)| = Phi(l,n) |Hyp(n)|                     (eq. MisCount)
* eta_l(k) = floor((l-1)/k) + 2                      (Thm fact_mis, eq. defMultHyp)
* sum_{k|n} (eta_l(k)|Hyp(k)| + sum_{j=2..l} |Mis(j,k)|) = 2^(l+n-1)   (eq. MisDeg)
"""


def divisors(n: int):
    return [k for k in range(1, n + 1) if n % k == 0]


def mobius(n: int) -> int:
    """Moebius function by trial division."""
    if n == 1:
        return 1
    res, m, p = 1, n, 2
    while p * p <= m:
        if m % p == 0:
            m //= p
            if m % p == 0:
                return 0
            res = -res
        p += 1
    if m > 1:
        res = -res
    return res


def hyp_count(n: int) -> int:
    """|Hyp(n)|: roots of p_n of exact period n."""
    return sum(mobius(n // k) * 2 ** (k - 1) for k in divisors(n))


def phi(l: int, n: int) -> int:
    """Phi(l, n) of eq. MisCount."""
    if l == 0:
        return 1
    if (l - 1) % n == 0:
        return 2 ** (l - 1) - 1
    return 2 ** (l - 1)


def mis_count(l: int, n: int) -> int:
    """|Mis(l,n)|; Mis(0,n) = Hyp(n) and Mis(1,n) is empty."""
    if l == 1:
        return 0
    return phi(l, n) * hyp_count(n)


def eta(l: int, k: int) -> int:
    """Multiplicity of Hyp(k) in q_{l,n} (k | n)."""
    return (l - 1) // k + 2


def degree(l: int, n: int) -> int:
    return 2 ** (l + n - 1)


def upper_half_count(total: int, n_real: int) -> int:
    """Number of roots stored in the closed upper half plane."""
    return n_real + (total - n_real) // 2
