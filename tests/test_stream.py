"""Streamed split of one type, chunk by chunk (msplit_split_streamed): p_n up
to n = 33, the paper's FP80 frontier (Section 6.3.2), with the level line cut
into seed ranges like the paper's independent jobs (Section 6.4.1).

CPU: the plan's host logic (workspace sizes, argument errors).  GPU: the
streamed split equals one pass of the same type (same count, same roots to
1e-12, same period labels) at sizes where one pass fits, with many chunks and
many real-part partitions; p_28 exercises the double-double tip starts of the
last chunk; p_31, p_32 and p_33 are checked by their exact per-period counts
(eq. HypCount), the certificate of every root and the oracle's long-double
certificate on a sample.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from oracle import counts


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# --------------------------------------------------------------------- CPU
def test_stream_workspace_sizes():
    from paper_2402_06083_amd import msplit
    ws = {n: msplit.stream_workspace_size(0, n) for n in (20, 28, 31, 32, 33)}
    # the accumulation (33 bytes per upper-half root and margin) plus one
    # chunk's workspace (2^28 starts by default)
    for n in (31, 32, 33):
        acc = 33 * msplit.stream_capacity(0, n)
        assert acc < ws[n] < acc + 40e9, (n, ws[n])
    assert ws[33] < 125e9
    # smaller chunks, smaller workspace
    assert msplit.stream_workspace_size(0, 31, chunk_starts=1 << 26) < ws[31]


@pytest.mark.parametrize("l,n,chunk", [(0, 34, 0), (1, 5, 0), (0, 0, 0), (2, 32, 0), (0, 20, 8), (0, 20, 1 << 31)])
def test_stream_argument_errors(l, n, chunk):
    from paper_2402_06083_amd import msplit
    with pytest.raises(msplit.MsplitError) as e:
        msplit.stream_workspace_size(l, n, chunk_starts=chunk)
    assert e.value.status in (msplit.E_ARG, msplit.E_PRECISION)


def test_stream_refuses_q_beyond_fp64():
    from paper_2402_06083_amd import msplit
    with pytest.raises(msplit.MsplitError) as e:
        msplit.stream_workspace_size(2, 26)
    assert e.value.status == msplit.E_PRECISION


# --------------------------------------------------------------------- GPU
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_06083_amd import msplit
    msplit.lib()
    return True


def _host(r):
    return r.cpu()


def _flagged(flags, bit, step=1 << 28):
    """Indices of the roots with a flag bit, slice by slice (torch.nonzero
    over more than 2^31 elements is not supported)."""
    out = [np.zeros(0, dtype=np.int64)]
    for s in range(0, flags.numel(), step):
        nz = torch.nonzero((flags[s:s + step] & bit) != 0).flatten()
        out.append(nz.cpu().numpy().astype(np.int64) + s)
    return np.concatenate(out)


def _period_hist(period, n):
    return {k: int((period == k).sum()) for k in range(1, n + 1) if n % k == 0}


def _check_full(g, st, n):
    """Exact per-period counts: roots of period k | n number |Hyp(k)|, each
    non-real one standing for its conjugate too."""
    real = g.im == 0
    for k in range(1, n + 1):
        if n % k:
            continue
        sel = g.period == k
        tot = int(real[sel].sum()) + 2 * int((~real[sel]).sum())
        assert tot == counts.hyp_count(k), (n, k, tot, counts.hyp_count(k))
    assert st["total"] == 2 ** (n - 1) and st["missing"] == 0, st


def _compare_one_pass(gs, g1):
    assert len(gs) == len(g1)
    assert np.array_equal(np.sort(gs.period), np.sort(g1.period))
    zs = gs.re + 1j * gs.im
    z1 = g1.re + 1j * g1.im
    from scipy.spatial import cKDTree
    tree = cKDTree(np.stack([g1.re, g1.im], axis=1))
    d, idx = tree.query(np.stack([gs.re, gs.im], axis=1), k=1)
    assert len(np.unique(idx)) == len(g1), "not a bijection"
    assert d.max() <= 1e-12, d.max()
    assert np.array_equal(gs.period, g1.period[idx])
    # the output is sorted by real part, as one pass
    assert np.all(np.diff(gs.re) >= -2.0 ** -45)
    return zs, z1


@pytest.mark.gpu
@pytest.mark.parametrize("n,chunk", [(12, 1 << 8), (20, 1 << 15), (24, 1 << 20)])
def test_streamed_equals_one_pass(gpu, n, chunk):
    """Many chunks (2^n / chunk of them) and many real-part partitions: the
    same certified roots as one pass of msplit_hyperbolic."""
    from paper_2402_06083_amd import msplit
    opts = msplit.make_options(certify=True)
    say(f"[gpu] streamed p_{n}, chunks of {chunk} starts")
    rs = msplit.split_streamed(0, n, opts, chunk_starts=chunk, check=False)
    torch.cuda.synchronize()
    st = rs.stats
    assert rs.status == msplit.OK, (rs.status, st)
    assert st["certified"] == len(rs) and st["label_proven"] == len(rs) and st["overlaps"] == 0, st
    assert st["discarded"] >= 0 and st["phase_fail"] == 0 and st["mark_capped"] == 0
    say(f"[gpu] one pass p_{n}")
    r1 = msplit.split(0, n, opts)
    torch.cuda.synchronize()
    gs, g1 = _host(rs), _host(r1)
    _compare_one_pass(gs, g1)
    _check_full(gs, st, n)
    assert st["starts"] == r1.stats["starts"] == 2 ** n + 1


@pytest.mark.gpu
def test_streamed_tip_starts_p28(gpu):
    """p_28 in 4 chunks: the double-double tip starts (last 4096 starts of the
    level line) sit in the last chunk; same roots as one pass, double-double
    roots to 1e-25."""
    from paper_2402_06083_amd import msplit
    opts = msplit.make_options(certify=True)
    say("[gpu] streamed p_28, chunks of 2^26 starts")
    rs = msplit.split_streamed(0, 28, opts, chunk_starts=1 << 26, check=False)
    torch.cuda.synchronize()
    st = rs.stats
    assert rs.status == msplit.OK, (rs.status, st)
    assert st["certified"] == len(rs) and st["overlaps"] == 0, st
    gs = _host(rs)
    del rs
    torch.cuda.empty_cache()
    say("[gpu] one pass p_28")
    r1 = msplit.split(0, 28, opts)
    torch.cuda.synchronize()
    g1 = _host(r1)
    del r1
    torch.cuda.empty_cache()
    _compare_one_pass(gs, g1)
    _check_full(gs, st, 28)
    dd = (gs.flags & msplit.R_DD) != 0
    assert dd.sum() > 0
    o = np.lexsort((g1.im, g1.re))
    s = np.lexsort((gs.im, gs.re))
    a, b = o[(g1.flags[o] & msplit.R_DD) != 0], s[(gs.flags[s] & msplit.R_DD) != 0]
    assert len(a) == len(b)
    err = np.abs((gs.re[b] - g1.re[a]) + (gs.re_lo[b] - g1.re_lo[a])) + \
        np.abs((gs.im[b] - g1.im[a]) + (gs.im_lo[b] - g1.im_lo[a]))
    assert err.max() < 1e-25, err.max()


@pytest.mark.gpu
@pytest.mark.parametrize("n", [31, 32, 33])
def test_streamed_frontier(gpu, n):
    """p_31 .. p_33 (2^30 .. 2^32 roots, the paper's FP80 frontier, Section
    6.3.2): exact counts per period, every root certified and its period
    proven, quarter-separated; the oracle's long-double certificate on a
    sample, double-double roots next to -2 included."""
    from paper_2402_06083_amd import msplit
    opts = msplit.make_options(certify=True)
    say(f"[gpu] streamed p_{n}")
    rs = msplit.split_streamed(0, n, opts, check=False)
    torch.cuda.synchronize()
    st = rs.stats
    say(f"[gpu] p_{n}: status {rs.status} count {len(rs)} ms {st['ms_device']:.0f} stages {st['ms_stage']} "
        f"dd {st['dd_routed']} discarded {st['discarded']} total {st['total']} real {st['n_real']} "
        f"overlaps {st['overlaps']} capped {st['mark_capped']} min_sep {st['min_sep']:.3g}")
    assert rs.status == msplit.OK, (rs.status, st)
    assert st["total"] == 2 ** (n - 1) and st["missing"] == 0, st
    assert st["certified"] == len(rs) and st["label_proven"] == len(rs) and st["overlaps"] == 0, st
    assert st["mark_capped"] == 0, st
    per = rs.period
    real = rs.im == 0
    for k in range(1, n + 1):
        if n % k == 0:
            sel = per == k
            tot = int((sel & real).sum().item()) + 2 * int((sel & ~real).sum().item())
            assert tot == counts.hyp_count(k), (n, k, tot)
    rng = np.random.default_rng(n)
    idx = np.sort(rng.choice(len(rs), size=3000, replace=False))
    dd = _flagged(rs.flags, msplit.R_DD)
    idx = np.unique(np.concatenate([idx, dd[:: max(1, len(dd) // 500)]]))
    it = torch.from_numpy(idx).to(rs.re.device)
    pick = lambda t: t[it].cpu().numpy()
    ok, rad = oracle.certify(0, n, pick(rs.re), pick(rs.im), pick(rs.re_lo), pick(rs.im_lo), pick(rs.period))
    assert np.all(ok == 3) and rad.max() <= 1e-10
    del rs
    torch.cuda.empty_cache()
