"""Helpers of the GPU parity tests: cached oracle splits and the comparison of
a GPU root list with the oracle's.

The bar (Thm certif reading, Section 6.2; nset identification, Section 6.1):
the same count, a nearest-neighbour bijection GPU -> oracle with every
distance <= 1e-10 and <= a quarter of the local root separation, identical
period labels and real flags; double-double roots (next to -2) agree with the
oracle's double-double values to 1e-25.
"""
import functools
import sys

import numpy as np

import oracle

TOL_ABS = 1e-10   # FP64 roots
TOL_DD = 1e-25    # double-double roots
R_DD = 8          # MSPLIT_R_DD


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def oracle_split(l, n, simple=False):
    say(f"[oracle] split l={l} n={n}{' simple' if simple else ''}")
    return oracle.split(l, n, simple=simple)


def compare_sets(g, o, tol=TOL_ABS, labels=True, dd_flags=None):
    """Nearest-neighbour bijection of the GPU roots g (re, im, period; and
    re_lo, im_lo with dd_flags) onto the oracle's o.  Returns dict(max_abs,
    max_over_sep, max_dd, idx): the largest distance, the largest distance
    over the local separation of the oracle root (its nearest other root or
    conjugate), the largest double-double error, and the matching."""
    from scipy.spatial import cKDTree
    oz = np.stack([o.re_hi, o.im_hi], axis=1)
    gz = np.stack([g.re, g.im], axis=1)
    assert len(gz) == len(oz), (len(gz), len(oz))
    if len(oz) == 0:
        return dict(max_abs=0.0, max_over_sep=0.0, max_dd=0.0, idx=np.zeros(0, dtype=np.int64))
    tree = cKDTree(oz)
    d, idx = tree.query(gz, k=1)
    assert len(np.unique(idx)) == len(oz), "not a bijection"
    if len(oz) > 1:
        dd, _ = tree.query(oz, k=2)
        sep = dd[:, 1]
    else:
        sep = np.full(1, np.inf)
    sep = np.minimum(sep, np.where(o.im_hi > 0, 2 * o.im_hi, np.inf))
    ratio = d / sep[idx]
    assert d.max() <= tol, d.max()
    assert np.all(ratio <= 0.25), ("a root moved by more than a quarter of its separation", ratio.max())
    if labels:
        assert np.array_equal(g.period, o.period[idx]), "period labels differ"
    assert np.array_equal(g.im == 0, o.im_hi[idx] == 0), "real flags differ"
    max_dd = 0.0
    if dd_flags is not None:
        sel = (dd_flags & R_DD) != 0
        if sel.any():
            ere = (g.re[sel] - o.re_hi[idx[sel]]) + (g.re_lo[sel] - o.re_lo[idx[sel]])
            eim = (g.im[sel] - o.im_hi[idx[sel]]) + (g.im_lo[sel] - o.im_lo[idx[sel]])
            max_dd = float(max(np.abs(ere).max(), np.abs(eim).max()))
            assert max_dd < TOL_DD, max_dd
    return dict(max_abs=float(d.max()), max_over_sep=float(ratio.max()), max_dd=max_dd, idx=idx)


class Host:
    """Host copies of one type's slice of a batch (the fields compare_sets
    reads)."""

    def __init__(self, runner, i):
        sl = runner.slices(i)
        self.re = runner.re[sl].cpu().numpy()
        self.im = runner.im[sl].cpu().numpy()
        self.re_lo = runner.re_lo[sl].cpu().numpy()
        self.im_lo = runner.im_lo[sl].cpu().numpy()
        self.period = runner.period[sl].cpu().numpy()
        self.preperiod = runner.preperiod[sl].cpu().numpy()
        self.flags = runner.flags[sl].cpu().numpy()
        self.radius = runner.radius[sl].cpu().numpy()

    def __len__(self):
        return len(self.re)
