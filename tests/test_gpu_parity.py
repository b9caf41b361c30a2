"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar (Section 6.1 / Thm certif reading): identical discrete structure -- same
root count, a nearest-neighbour bijection with every distance <= 1e-10 and
<= a quarter of the local root separation, identical period labels and real
flags.  At the full period-24 size every returned root is checked one by one
by the oracle's own certificate (Thm proofRoots in long double) on a sample,
and by the GPU certificate plus exact counts on all of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import counts
from parity import compare_sets, oracle_split, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_06083_amd import msplit
    msplit.lib()  # raises if the HIP library is missing
    return torch.device("cuda:0")


def gpu_split(l, n, **kw):
    from paper_2402_06083_amd import msplit
    say(f"[gpu] split l={l} n={n} {kw}")
    opts = msplit.make_options(**kw)
    r = msplit.split(l, n, opts, check=False)
    torch.cuda.synchronize()
    return r, r.cpu()


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_hyperbolic_parity_small(n):
    from paper_2402_06083_amd import msplit
    r, g = gpu_split(0, n)
    assert r.status == msplit.OK, (r.status, r.stats)
    st = r.stats
    assert st["phase_fail"] == 0 and st["missing"] == 0 and st["total"] == 2 ** (n - 1)
    o = oracle_split(0, n)
    compare_sets(g, o)
    # increasing real part
    assert np.all(np.diff(g.re) >= -2.0 ** -45)  # ordered to the key resolution 2^-46


@pytest.mark.parametrize("n,seg_points,ppt", [(12, 2, 8), (12, 4, 8), (14, 1024, 8), (12, 4, 16), (13, 2, 16)])
def test_segment_lengths_match_oracle(n, seg_points, ppt):
    """Segments from the shortest (one start: the two walks of a segment meet
    on it, and their meeting points need a buffer of their own) to the
    longest, with 8 and 16 points per turn: the same root set as the
    oracle, every root certified, no failed phase check."""
    from paper_2402_06083_amd import msplit
    r, g = gpu_split(0, n, seg_points=seg_points, points_per_turn=ppt, certify=True)
    assert r.status == msplit.OK, (r.status, r.stats)
    st = r.stats
    assert st["phase_fail"] == 0 and st["missing"] == 0 and st["certified"] == st["unique"], st
    compare_sets(g, oracle_split(0, n))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hyperbolic_parity_n20(precision):
    from paper_2402_06083_amd import msplit
    r, g = gpu_split(0, 20, precision=precision)
    assert r.status == msplit.OK, (r.status, r.stats)
    o = oracle_split(0, 20)
    dmax = compare_sets(g, o)["max_abs"]
    say(f"[gpu] n=20 {precision}: max |gpu - oracle| = {dmax:.3e}, stats={r.stats}")
    if precision == "mixed":
        assert r.stats["steps_fp32"] > 0


@pytest.mark.parametrize("n", [12, 18])
def test_certificate_on_split(n):
    from paper_2402_06083_amd import msplit
    r, g = gpu_split(0, n, certify=True)
    assert r.status == msplit.OK
    st = r.stats
    assert st["certified"] == len(g) and st["label_proven"] == len(g), st
    assert st["overlaps"] == 0
    assert np.all(g.flags & msplit.R_CERTIFIED) and np.all(g.flags & msplit.R_LABEL)
    assert g.radius.max() <= 1e-10
    # the oracle's certificate (long double, round upward) accepts them too
    ok, rad = oracle.certify(0, n, g.re, g.im, label=g.period)
    assert np.all(ok == 3)


def check_full_period(n, sample=4000, seed=0):
    """p_n at full size: exact counts per period class (eq. HypCount) taken on
    the device, every root certified with its period proven, no overlap, and a
    random sample -- with the double-double roots next to -2 -- certified again
    by the oracle from the double-double values."""
    from paper_2402_06083_amd import msplit
    opts = msplit.make_options(certify=True)
    b = msplit.Buffers(0, n, opts)
    r = msplit.split(0, n, opts, buffers=b, check=False)
    torch.cuda.synchronize()
    st = r.stats
    say(f"[gpu] p_{n}: status {r.status} stages {st['ms_stage']} dd_routed {st['dd_routed']}")
    assert r.status == msplit.OK, (r.status, st)
    assert st["total"] == 2 ** (n - 1) and st["certified"] == len(r) and st["label_proven"] == len(r), st
    assert st["overlaps"] == 0 and st["max_radius"] <= 1e-10, st
    for k in counts.divisors(n):
        sel = r.period == k
        cnt = int((r.im[sel] == 0).sum().item()) + 2 * int((r.im[sel] > 0).sum().item())
        assert cnt == counts.hyp_count(k), (k, cnt)
    dd = torch.nonzero((r.flags & msplit.R_DD) != 0).flatten()
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(len(r), size=sample, replace=False))
    idx = np.union1d(idx, dd[: min(len(dd), 200)].cpu().numpy())
    t = torch.as_tensor(idx, device=r.re.device)
    ok, rad = oracle.certify(0, n, r.re[t].cpu().numpy(), r.im[t].cpu().numpy(), r.re_lo[t].cpu().numpy(),
                             r.im_lo[t].cpu().numpy(), label=r.period[t].cpu().numpy())
    assert np.all(ok == 3) and rad.max() <= 1e-10
    del b, r
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [25, 26])
def test_full_size_beyond_fp64(n):
    """p_25, p_26: past the FP64 separation of the roots next to -2
    (118.4 / 4^n, Section 6.3.2); the tip goes through double-double."""
    check_full_period(n, seed=n)


def test_full_size_period_28():
    check_full_period(28, seed=28)


def test_full_size_period_30():
    """p_30 (536 870 912 roots), the double-double storage configuration:
    the starts at the left tip are re-solved in double-double."""
    check_full_period(30, sample=2000, seed=30)


def test_full_size_period_24():
    """Period 24 at full size (8 388 608 roots): exact counts per period class,
    every root certified by the GPU, a random sample certified one by one by
    the oracle, Vieta's sum of the roots."""
    from paper_2402_06083_amd import msplit
    n = 24
    r, g = gpu_split(0, n, certify=True)
    assert r.status == msplit.OK, (r.status, r.stats)
    st = r.stats
    say(f"[gpu] n=24 stats: {st}")
    assert st["total"] == 2 ** 23 and st["certified"] == len(g) and st["label_proven"] == len(g)
    assert st["overlaps"] == 0 and g.radius.max() <= 1e-10
    for k in counts.divisors(n):
        sel = g.period == k
        cnt = int((g.im[sel] == 0).sum()) + 2 * int((g.im[sel] > 0).sum())
        assert cnt == counts.hyp_count(k), (k, cnt)
    rng = np.random.default_rng(24)
    idx = rng.choice(len(g), size=20000, replace=False)
    idx.sort()
    ok, rad = oracle.certify(0, n, g.re[idx], g.im[idx], label=g.period[idx])
    assert np.all(ok == 3)
    assert rad.max() <= 1e-10
    w = np.where(g.im > 0, 2.0, 1.0)
    s1 = math.fsum((w * g.re).tolist())
    assert abs(s1 - (-(2 ** (n - 2)))) < 1e-6


def test_batch_periods_1_to_24_default_options():
    """All periods 1..24 through msplit_batch with the default launch options
    (the tuned options of the benchmark are compared with the oracle in
    test_gpu_oracle_exact): exact counts, every root certified with its
    period proven, radius <= 1e-10, quarter-separated."""
    from paper_2402_06083_amd import batch
    say("[gpu] batch 1..24, default options")
    res = batch.run_batch([(0, n) for n in range(1, 25)], certify=True)
    for (l, n), (count, st, status) in zip(res.pairs, res.per_pair):
        assert status == 0, (n, status, st)
        assert st["total"] == 2 ** (n - 1) and st["certified"] == count and st["overlaps"] == 0, (n, st)
        assert st["label_proven"] == count and st["max_radius"] <= 1e-10, (n, st)


# q_{l,n}: preperiods 2..15, periods 1..13, orders 3..16
MIS_SMALL = [(2, 1), (2, 2), (3, 1), (2, 3), (3, 2), (4, 2), (2, 5), (3, 4), (5, 3), (2, 8), (4, 6), (8, 4),
             (12, 2), (2, 12), (6, 8), (13, 1), (10, 6), (3, 13), (15, 1), (7, 7)]


@pytest.mark.parametrize("ln", MIS_SMALL)
def test_misiurewicz_parity_small(ln):
    """Mis(l,n) (eq. def:mis): the same set as the oracle, exact count
    (eq. MisCount), period n and preperiod l on every root."""
    from paper_2402_06083_amd import msplit
    l, n = ln
    r, g = gpu_split(l, n)
    assert r.status == msplit.OK, (r.status, r.stats)
    st = r.stats
    assert st["phase_fail"] == 0 and st["missing"] == 0 and st["total"] == counts.mis_count(l, n), st
    o = oracle_split(l, n)
    compare_sets(g, o)
    assert np.all(g.period == n) and np.all(g.preperiod == l)
    assert np.all(np.diff(g.re) >= -2.0 ** -45)  # ordered to the key resolution 2^-46


@pytest.mark.parametrize("ln", [(2, 10), (5, 7), (11, 3)])
def test_misiurewicz_certificate(ln):
    """Every returned root certified with its type proven on the disk (no
    root of q_{l-1,n} or of q_{l,k}, k | n, k < n); the oracle's long-double
    certificate accepts the same disks' centres."""
    from paper_2402_06083_amd import msplit
    l, n = ln
    r, g = gpu_split(l, n, certify=True)
    assert r.status == msplit.OK, (r.status, r.stats)
    st = r.stats
    assert st["certified"] == len(g) and st["label_proven"] == len(g) and st["overlaps"] == 0, st
    assert g.radius.max() <= 1e-10
    ok, rad = oracle.certify(l, n, g.re, g.im)
    assert np.all(ok == 3)


def mis_pairs(max_order):
    return [(l, s - l) for s in range(3, max_order + 1) for l in range(2, s)]


@pytest.mark.parametrize("ln", [(3, 15), (6, 13), (2, 16), (4, 14)])
def test_misiurewicz_parity_tip(ln):
    """Orders 18 and 19: real Misiurewicz parameters next to -2 pair up below
    1e-12 and q_{l,n} has centres of high multiplicity (Thm fact_mis) that
    stall descents.  Same set as the oracle, exact count; the double-double
    roots (MSPLIT_R_DD) agree with the oracle's to 1e-25."""
    from paper_2402_06083_amd import msplit
    l, n = ln
    r, g = gpu_split(l, n, certify=True)
    st = r.stats
    assert r.status == msplit.OK, (r.status, st)
    assert st["total"] == counts.mis_count(l, n) and st["certified"] == len(g) and st["overlaps"] == 0, st
    assert st["dd_routed"] > 0
    o = oracle_split(l, n)
    idx = compare_sets(g, o)["idx"]
    dd = (g.flags & msplit.R_DD) != 0
    assert dd.any()
    ere = (g.re[dd] - o.re_hi[idx[dd]]) + (g.re_lo[dd] - o.re_lo[idx[dd]])
    eim = (g.im[dd] - o.im_hi[idx[dd]]) + (g.im_lo[dd] - o.im_lo[idx[dd]])
    assert np.max(np.abs(ere)) < 1e-25 and np.max(np.abs(eim)) < 1e-25


def test_certify_api_and_rejection():
    from paper_2402_06083_amd import msplit
    o = oracle_split(0, 12)
    say("[gpu] msplit_certify on oracle roots")
    re = torch.tensor(o.re_hi, dtype=torch.float64, device="cuda")
    im = torch.tensor(o.im_hi, dtype=torch.float64, device="cuda")
    per = torch.tensor(o.period, dtype=torch.int32, device="cuda")
    flags, rad, st = msplit.certify(0, 12, re, im, per)
    f = flags.cpu().numpy()
    assert np.all(f & msplit.R_CERTIFIED) and np.all(f & msplit.R_LABEL)
    assert st["overlaps"] == 0
    # a candidate moved by 1e-3 is not certified within 1e-10, a wrong label fails
    re2 = re.clone()
    re2[100] += 1e-3
    per2 = per.clone()
    j = int(np.where(o.period == 12)[0][5])
    per2[j] = 6
    flags, rad, st = msplit.certify(0, 12, re2, im, per2)
    f = flags.cpu().numpy()
    r = rad.cpu().numpy()
    assert not (f[100] & msplit.R_CERTIFIED and r[100] <= 1e-10)
    assert (f[j] & msplit.R_CERTIFIED) and not (f[j] & msplit.R_LABEL)


def test_error_paths():
    import ctypes
    from paper_2402_06083_amd import msplit
    L = msplit.lib()
    opts = msplit.make_options()
    say("[gpu] error paths")
    ws_bytes = msplit.workspace_size(0, 10, opts)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    cap = 10
    re = torch.empty(cap, dtype=torch.float64, device="cuda")
    im = torch.empty(cap, dtype=torch.float64, device="cuda")
    rs = msplit.RootsC(re.data_ptr(), im.data_ptr(), None, None, None, None, None, None, cap)
    cnt = ctypes.c_uint64()
    st = msplit.Stats()
    sh = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    r = L.msplit_hyperbolic(10, ctypes.byref(opts), ctypes.c_void_p(ws.data_ptr()), ws_bytes, ctypes.byref(rs),
                            ctypes.byref(cnt), ctypes.byref(st), sh)
    assert r == msplit.E_CAPACITY and cnt.value == len(oracle_split(0, 10))
    r = L.msplit_hyperbolic(10, ctypes.byref(opts), ctypes.c_void_p(ws.data_ptr()), ws_bytes - 4096,
                            ctypes.byref(rs), ctypes.byref(cnt), ctypes.byref(st), sh)
    assert r == msplit.E_WORKSPACE
    # q_{4,22}: tau of order 26 is below the FP64 floor (no double-double route for q there)
    r = L.msplit_misiurewicz(4, 22, ctypes.byref(opts), ctypes.c_void_p(ws.data_ptr()), ws_bytes,
                             ctypes.byref(rs), ctypes.byref(cnt), ctypes.byref(st), sh)
    assert r == msplit.E_PRECISION


def _batch_snapshot(runner):
    out = []
    for i in range(len(runner.pairs)):
        sl = runner.slices(i)
        out.append(tuple(t[sl].cpu().numpy().copy() for t in (runner.re, runner.im, runner.re_lo, runner.im_lo,
                                                               runner.period, runner.flags, runner.radius)))
    return [int(c) for c in runner.counts], out


def test_batch_graph_replays_match_eager():
    """msplit_batch_graph: the captured batch (periods 1..16 and three
    Misiurewicz types, one with the double-double route) replayed three
    times, with eager work and synchronisations between the replays; every
    replay equals the eager call bit for bit."""
    from paper_2402_06083_amd import batch, msplit
    pairs = [(0, n) for n in range(1, 17)] + [(2, 5), (3, 4), (4, 10)]
    opts = msplit.make_options(certify=True)
    runner = batch.BatchRunner(pairs, opts)
    say("[gpu] graph: eager reference")
    r = runner.run()
    torch.cuda.synchronize()
    assert r == 0, msplit.strerror(r)
    ref_counts, ref = _batch_snapshot(runner)
    ref_stats = [s.as_dict() for s in runner.stats]
    for (l, n), c, st in zip(pairs, ref_counts, ref_stats):
        assert st["certified"] == c and st["missing"] == 0, (l, n, st)
    say("[gpu] graph: capture")
    runner.capture()
    x = torch.arange(1 << 20, device="cuda", dtype=torch.float64)
    for rep in range(3):
        say(f"[gpu] graph: replay {rep}")
        runner.re.fill_(float("nan"))
        runner.radius.zero_()
        torch.cuda.synchronize()
        r = runner.launch()
        assert r == 0, msplit.strerror(r)
        counts, snap = _batch_snapshot(runner)
        assert counts == ref_counts
        for i, (a, b) in enumerate(zip(snap, ref)):
            for u, v in zip(a, b):
                assert np.array_equal(u, v, equal_nan=True), (pairs[i], rep)
        st = [s.as_dict() for s in runner.stats]
        assert [s["certified"] for s in st] == [s["certified"] for s in ref_stats]
        # eager work between the replays
        y = (x * 3.0).sum()
        torch.cuda.synchronize()
        assert float(y) == 3.0 * (1 << 20) * ((1 << 20) - 1) / 2
    runner.close()


def test_misiurewicz_batch_mixed_precision():
    """MIXED precision on Misiurewicz types (their descents run in FP64 from
    the start) and p_n types in one batch: complete and certified."""
    from paper_2402_06083_amd import batch
    pairs = [(0, 16), (2, 8), (3, 11), (6, 6), (5, 12)]
    say("[gpu] mixed batch with Misiurewicz types")
    res = batch.run_batch(pairs, certify=True, precision="mixed")
    for (l, n), (count, st, status) in zip(res.pairs, res.per_pair):
        assert status == 0 and st["missing"] == 0 and st["certified"] == count, (l, n, st)
        assert st["total"] == counts.mis_count(l, n) if l else st["total"] == 2 ** (n - 1)


def test_mixed_batch_equals_fp64_eligible_types_interleaved():
    """MIXED on a batch whose FP32-eligible types (p_n, n <= 20) lie between
    types without an FP32 pass (p_21, q_{l,n}): the FP32 pass runs over the
    eligible starts alone (its own index space), the others descend in FP64
    from the walk's first iterate; per type the same certified roots as the
    FP64 run (same count and period labels, roots within 1e-12), FP32 steps
    on the eligible types only."""
    from paper_2402_06083_amd import batch, msplit
    pairs = [(0, 21), (0, 12), (3, 9), (0, 9), (2, 10), (0, 17)]
    runs = {}
    for prec in ("fp64", "mixed"):
        say(f"[gpu] interleaved batch {prec}")
        opts = msplit.make_options(precision=prec, certify=True, fp32_switch=2.0 ** -4)
        r = batch.BatchRunner(pairs, opts)
        assert r.run() == 0
        torch.cuda.synchronize()
        runs[prec] = r
    for i, (l, n) in enumerate(pairs):
        a, b = runs["fp64"], runs["mixed"]
        sa, sb = a.stats[i].as_dict(), b.stats[i].as_dict()
        assert sa["missing"] == sb["missing"] == 0 and sb["certified"] == int(b.counts[i]), (l, n, sb)
        assert int(a.counts[i]) == int(b.counts[i]), (l, n)
        eligible = l == 0 and n <= 20
        assert (sb["steps_fp32"] > 0) == eligible and sa["steps_fp32"] == 0, (l, n, sb["steps_fp32"])
        za, zb = a.slices(i), b.slices(i)
        ra, ia = a.re[za].cpu().numpy(), a.im[za].cpu().numpy()
        rb, ib = b.re[zb].cpu().numpy(), b.im[zb].cpu().numpy()
        oa, ob = np.lexsort((ia, ra)), np.lexsort((ib, rb))
        d = np.abs((ra[oa] - rb[ob]) + 1j * (ia[oa] - ib[ob]))
        assert d.max() <= 1e-12, (l, n, d.max())
        assert np.array_equal(a.period[za].cpu().numpy()[oa], b.period[zb].cpu().numpy()[ob]), (l, n)
    for r in runs.values():
        r.close()


def test_autotuner_picks_a_complete_configuration(tmp_path):
    """The autotuner times candidate launch parameters on a batch, rejects
    incomplete splits and caches the fastest; the cached options split the
    batch completely (every root certified)."""
    from paper_2402_06083_amd import batch, msplit, tune
    pairs = [(0, n) for n in range(1, 15)] + [(3, 9)]
    path = str(tmp_path / "tune.json")
    say("[gpu] autotune")
    res = tune.tune(pairs, "fp64", space={"block_size": [128, 256], "seg_points": [0, 64],
                                           "points_per_turn": [8, 16]}, path=path)
    assert len(res["trials"]) == 9 and all("ms" in t for t in res["trials"]), res["trials"]
    hit = tune.lookup(pairs, "fp64", path=path)
    assert hit is not None and hit["options"] == res["best"]
    opts, cand = tune.tuned_options(pairs, "fp64", path=path)
    assert cand == res["best"]
    runner = batch.BatchRunner(pairs, opts)
    r = runner.run()
    torch.cuda.synchronize()
    assert r == 0, msplit.strerror(r)
    for (l, n), s in zip(pairs, runner.stats):
        d = s.as_dict()
        assert d["missing"] == 0 and d["certified"] == d["unique"], (l, n, d)


@pytest.mark.parametrize("ln", [(0, 14), (3, 9), (2, 16)])
def test_basin_radii_verified_by_oracle(ln):
    """MSPLIT_F_BASIN (Thm proofContract): every certified root gets a disk of
    Newton convergence; the oracle re-proves each claim (root within
    radius + |lo| of the FP64 centre, basin disk) in long-double disk
    arithmetic, and no basin disk reaches another root.  (2,16) includes
    double-double roots next to -2."""
    from paper_2402_06083_amd import msplit
    l, n = ln
    r, g = gpu_split(l, n, certify=True, basin=True)
    st = r.stats
    assert st["certified"] == len(g) and st["basin"] == len(g), st
    assert np.all(g.flags & msplit.R_BASIN)
    assert np.all(g.basin > 0) and st["min_basin"] == g.basin.min()
    eta = g.radius + np.abs(g.re_lo) + np.abs(g.im_lo)
    assert np.all(oracle.basin_check(l, n, g.re, g.im, eta, g.basin))
    z = (g.re + g.re_lo) + 1j * (g.im + g.im_lo)
    allz = np.concatenate([z, np.conj(z[g.im > 0])])
    from scipy.spatial import cKDTree
    tree = cKDTree(np.stack([allz.real, allz.imag], axis=1))
    d, _ = tree.query(np.stack([z.real, z.imag], axis=1), k=2)
    assert np.all(g.basin < d[:, 1])


def test_certify_api_basin():
    """msplit_certify with a basin array: the same radii as the split."""
    from paper_2402_06083_amd import msplit
    r, g = gpu_split(0, 10, certify=True, basin=True)
    flags, radius, st, bas = msplit.certify(0, 10, r.re, r.im, period=r.period, basin=True)
    torch.cuda.synchronize()
    assert st["basin"] == len(g)
    assert np.array_equal(bas.cpu().numpy(), g.basin)
    assert np.array_equal(flags.cpu().numpy() & msplit.R_BASIN, g.flags & msplit.R_BASIN)


# ---------------------------------------------------------------------------
# Mis(l,n) from the simplified polynomial s_{l,n} = p_{l+n-1} + p_{l-1}
# (eq. polySimple, MSPLIT_F_SIMPLE): the same set as the q_{l,n} route and as
# the oracle's s route, from half as many starts.

def oracle_split_simple(l, n):
    return oracle_split(l, n, simple=True)


SIMPLE_SMALL = [(2, 1), (3, 1), (2, 2), (4, 2), (3, 4), (5, 3), (2, 8), (7, 2), (4, 6), (9, 3), (12, 2), (6, 8),
                (3, 12), (13, 2), (5, 10)]


@pytest.mark.parametrize("ln", SIMPLE_SMALL)
def test_simple_parity_small(ln):
    """s_{l,n} route: exact count |Mis(l,n)|, start count 2^(l+n-1) + 1 (half
    the q route's), the oracle's s-route set, and the oracle's q-route set."""
    from paper_2402_06083_amd import msplit
    l, n = ln
    r, g = gpu_split(l, n, simple=True)
    assert r.status == msplit.OK, (r.status, r.stats)
    st = r.stats
    assert st["phase_fail"] == 0 and st["missing"] == 0 and st["total"] == counts.mis_count(l, n), st
    assert st["starts"] == 2 ** (l + n - 1) + 1, st
    compare_sets(g, oracle_split_simple(l, n))
    compare_sets(g, oracle_split(l, n))
    assert np.all(g.period == n) and np.all(g.preperiod == l)


@pytest.mark.parametrize("ln", [(2, 10), (5, 7), (3, 15), (2, 16)])
def test_simple_certified(ln):
    """s_{l,n} route with the certificate (Thm proofRoots on q_{l,n}): every
    root certified with its type proven; at orders 18 and 19 (the tip next to
    -2 in double-double) the set equals the oracle's q-route set."""
    from paper_2402_06083_amd import msplit
    l, n = ln
    r, g = gpu_split(l, n, certify=True, simple=True)
    st = r.stats
    assert r.status == msplit.OK, (r.status, st)
    assert st["total"] == counts.mis_count(l, n), st
    assert st["certified"] == len(g) and st["label_proven"] == len(g) and st["overlaps"] == 0, st
    o = oracle_split(l, n)
    compare_sets(g, o)
    rng = np.random.default_rng(l * 100 + n)
    idx = np.sort(rng.choice(len(g), size=min(2000, len(g)), replace=False))
    ok, rad = oracle.certify(l, n, g.re[idx], g.im[idx], g.re_lo[idx], g.im_lo[idx])
    assert np.all(ok == 3) and rad.max() <= 1e-10


@pytest.mark.parametrize("ln", [(2, 6), (5, 4), (3, 11)])
def test_simple_starts_on_level_line(ln):
    """Start k of the s route has s_{l,n} = lambda_0 i^k (level 100), checked by
    the oracle's long-double evaluation of s_{l,n}."""
    from paper_2402_06083_amd import msplit
    l, n = ln
    say(f"[gpu] starts s l={l} n={n}")
    re, im, st, status = msplit.starts(l, n, msplit.make_options(simple=True), check=False)
    assert status == msplit.OK and st["phase_fail"] == 0, st
    g = re.cpu().numpy() + 1j * im.cpu().numpy()
    assert len(g) == 2 ** (l + n - 1) + 1
    for k in range(0, len(g), max(1, len(g) // 64)):
        P = oracle.evaluate(l, n, complex(g[k]), simple=True)
        val = complex(float(P[0]), float(P[1]))
        assert abs(val / (100 * [1, 1j, -1, -1j][k % 4]) - 1) < 2 ** -5 + 1e-9, k


def test_simple_batch_all_pairs():
    """All 210 types with l + n <= 22 through the s route in one certified
    batch: exact counts per pair, every root certified, and per pair the same
    roots as the q-route batch (sorted real parts agree to 1e-12)."""
    from paper_2402_06083_amd import batch
    pairs = mis_pairs(22)
    say("[gpu] batch of all s_{l,n}, l + n <= 22")
    rs = batch.run_batch(pairs, certify=True, simple=True)
    rq = batch.run_batch(pairs, certify=True)
    for i, ((l, n), (count, st, status)) in enumerate(zip(rs.pairs, rs.per_pair)):
        assert status == 0, ((l, n), status, st)
        assert st["total"] == counts.mis_count(l, n), ((l, n), st)
        assert st["certified"] == count and st["label_proven"] == count and st["overlaps"] == 0, ((l, n), st)
        assert count == rq.per_pair[i][0], (l, n)
        zs = rs.bufs.re[rs.bufs.slices(i)].cpu().numpy() + 1j * rs.bufs.im[rs.bufs.slices(i)].cpu().numpy()
        zq = rq.bufs.re[rq.bufs.slices(i)].cpu().numpy() + 1j * rq.bufs.im[rq.bufs.slices(i)].cpu().numpy()
        zs, zq = np.sort_complex(zs), np.sort_complex(zq)
        assert np.max(np.abs(zs - zq)) <= 1e-12, (l, n)


def test_deterministic_output():
    r1, g1 = gpu_split(0, 17)
    r2, g2 = gpu_split(0, 17)
    assert np.array_equal(g1.re, g2.re) and np.array_equal(g1.im, g2.im)
    assert np.array_equal(g1.period, g2.period)


@pytest.mark.parametrize("n", [3, 8, 12, 17])
def test_start_set_matches_oracle(n):
    """Start k of the GPU level line is the oracle's start k (value lambda_0 i^k),
    up to the acceptance tolerance of the walk."""
    from paper_2402_06083_amd import msplit
    say(f"[gpu] starts n={n}")
    re, im, st, status = msplit.starts(0, n, check=False)
    assert status == msplit.OK and st["phase_fail"] == 0, st
    g = re.cpu().numpy() + 1j * im.cpu().numpy()
    ore, oim, _ = oracle.starts(0, n)
    o = ore.astype(np.float64) + 1j * oim.astype(np.float64)
    assert len(g) == len(o) == 2 ** n + 1
    gap = np.minimum(np.abs(np.diff(o, prepend=o[1])), np.abs(np.diff(o, append=o[-2])))
    assert np.all(np.abs(g - o) <= 0.2 * gap)
    for k in range(0, len(g), max(1, len(g) // 50)):
        P = oracle.evaluate(0, n, complex(g[k]))
        val = complex(float(P[0]), float(P[1]))
        assert abs(val / (5 * [1, 1j, -1, -1j][k % 4]) - 1) < 2 ** -5 + 1e-9, k
