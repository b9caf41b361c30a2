"""msplit_hyperbolic_static, the entry point that allocates nothing (its
workspace is the library's static device array), against msplit_hyperbolic
on the same inputs: two calls in a row, the second with a smaller input,
each equal to the workspace entry point root by root (the same kernels on
the same inputs: the same bits), and the whole output set against the
oracle."""
import ctypes
import sys

import numpy as np
import pytest

from parity import compare_sets, oracle_split, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_06083_amd import msplit
    msplit.lib()
    return torch.device("cuda:0")


def _host(r):
    g = r.cpu()
    return g


@pytest.mark.parametrize("certify", [True, False])
def test_static_entry_point_equals_workspace_entry_point(certify):
    from paper_2402_06083_amd import msplit
    for n in (18, 12):  # the second call smaller: the array keeps the first call's contents
        opts = msplit.make_options(certify=certify)
        say(f"[gpu] p_{n} through msplit_hyperbolic_static (certify={certify})")
        rs = msplit.hyperbolic_static(n, opts, check=False)
        torch.cuda.synchronize()
        assert rs.status == msplit.OK, (rs.status, rs.stats)
        say(f"[gpu] p_{n} through msplit_hyperbolic")
        rw = msplit.split(0, n, opts, check=False)
        torch.cuda.synchronize()
        assert rw.status == msplit.OK, (rw.status, rw.stats)
        gs, gw = _host(rs), _host(rw)
        assert len(gs) == len(gw) and rs.stats["total"] == rw.stats["total"] == 2 ** (n - 1)
        for k in ("re", "im", "period", "flags", "re_lo", "im_lo"):
            assert np.array_equal(getattr(gs, k), getattr(gw, k)), (n, k)
        if certify:
            assert np.array_equal(gs.radius, gw.radius)
            assert rs.stats["certified"] == len(gs) and rs.stats["overlaps"] == 0
        for k in ("unique", "n_real", "converged", "steps_desc", "steps_walk", "sorted"):
            assert rs.stats[k] == rw.stats[k], k
        assert rs.stats["ms_device"] == 0.0
        compare_sets(gs, oracle_split(0, n))


def test_static_entry_point_refuses_beyond_its_array():
    """p_20 needs more than MSPLIT_STATIC_SCRATCH_BYTES: MSPLIT_E_WORKSPACE,
    count 0, and the next call still works."""
    from paper_2402_06083_amd import msplit
    opts = msplit.make_options()
    b = msplit.Buffers(0, 20, opts, ws_bytes=0)
    r = msplit.hyperbolic_static(20, opts, buffers=b, check=False)
    assert r.status == msplit.E_WORKSPACE and r.count == 0
    r = msplit.hyperbolic_static(10, opts, check=False)
    torch.cuda.synchronize()
    assert r.status == msplit.OK and r.count > 0
