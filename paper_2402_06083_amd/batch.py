"""Batched splits through ``msplit_batch`` with preallocated device buffers.

The benchmark and the batch parity test share this runner so that both use the
same launch configuration.
"""
import ctypes

import torch

from . import msplit


# the stated accuracy of a certified root: the radius of its unique-root disk
RADIUS_MAX = 1e-10


def unproven(st, certify=True, labels=True):
    """Why a type's split does not prove its root set (empty when it does).
    By Thm certif (Section 6.2) the list is the root set when every root has
    a disk holding exactly one root of P, the disks are pairwise disjoint
    (here quarter-separated) and the count equals the degree (|Mis(l,n)| for
    q_{l,n}); the stated accuracy is radius <= 1e-10."""
    why = []
    if st["missing"] or st["total"] != st["expected"]:
        why.append(f"count {st['total']} of {st['expected']}")
    if certify:
        if st["certified"] != st["unique"]:
            why.append(f"certified {st['certified']} of {st['unique']}")
        if labels and st["label_proven"] != st["unique"]:
            why.append(f"labels proven {st['label_proven']} of {st['unique']}")
        if st["overlaps"]:
            why.append(f"{st['overlaps']} disks not quarter-separated")
        if not st["max_radius"] <= RADIUS_MAX:
            why.append(f"radius {st['max_radius']:.3g} > {RADIUS_MAX:g}")
    return why


class BatchResult:
    def __init__(self, pairs, caps, counts, stats, statuses, bufs):
        self.pairs = pairs
        self.caps = caps
        self.per_pair = list(zip(counts, stats, statuses))
        self.bufs = bufs


class BatchRunner:
    """Buffers sized once for a list of (l, n) pairs; ``run()`` splits all."""

    def __init__(self, pairs, opts, device="cuda"):
        self.pairs = list(pairs)
        self.opts = opts
        L = msplit.lib()
        self.arr = (ctypes.c_int32 * (2 * len(self.pairs)))(*[v for p in self.pairs for v in p])
        b = ctypes.c_uint64()
        r = L.msplit_batch_workspace_size(self.arr, len(self.pairs), ctypes.byref(opts), ctypes.byref(b))
        if r:
            raise msplit.MsplitError(r, "msplit_batch_workspace_size")
        self.ws_bytes = int(b.value)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        # capacity per pair: all roots of q_{l,n} fit in 2^(l+n-1) upper-half slots
        self.caps = [1 << (l + n - 1) for (l, n) in self.pairs]
        tot = sum(self.caps)
        self.re = torch.empty(tot, dtype=torch.float64, device=device)
        self.im = torch.empty(tot, dtype=torch.float64, device=device)
        self.re_lo = torch.empty(tot, dtype=torch.float64, device=device)
        self.im_lo = torch.empty(tot, dtype=torch.float64, device=device)
        self.period = torch.empty(tot, dtype=torch.int32, device=device)
        self.preperiod = torch.empty(tot, dtype=torch.int32, device=device)
        self.flags = torch.empty(tot, dtype=torch.uint8, device=device)
        self.radius = torch.empty(tot, dtype=torch.float64, device=device)
        self.basin = torch.empty(tot, dtype=torch.float64, device=device) if opts.flags & msplit.F_BASIN else None
        self.caps_arr = (ctypes.c_uint64 * len(self.pairs))(*self.caps)
        self.counts = (ctypes.c_uint64 * len(self.pairs))()
        self.stats = (msplit.Stats * len(self.pairs))()
        self.roots = msplit.RootsC(self.re.data_ptr(), self.im.data_ptr(), self.re_lo.data_ptr(),
                                   self.im_lo.data_ptr(), self.period.data_ptr(),
                                   self.preperiod.data_ptr(), self.flags.data_ptr(), self.radius.data_ptr(), tot,
                                   self.basin.data_ptr() if self.basin is not None else None)

        self._graph = None
        self._gstream = None

    def run(self, stream=None):
        L = msplit.lib()
        sh = msplit._stream_handle(stream)
        r = L.msplit_batch(self.arr, len(self.pairs), ctypes.byref(self.opts), ctypes.c_void_p(self.ws.data_ptr()),
                           self.ws_bytes, ctypes.byref(self.roots), self.caps_arr, self.counts, self.stats, sh)
        return r

    def capture(self):
        """Capture the batch as one hipGraph (msplit_batch_graph) on a stream of
        its own (the null stream cannot be captured)."""
        if self._graph is not None:
            return
        L = msplit.lib()
        self._gstream = torch.cuda.Stream(device=self.ws.device)
        torch.cuda.synchronize()
        g = ctypes.c_void_p()
        r = L.msplit_batch_graph(self.arr, len(self.pairs), ctypes.byref(self.opts),
                                 ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, ctypes.byref(self.roots),
                                 self.caps_arr, ctypes.c_void_p(self._gstream.cuda_stream), ctypes.byref(g))
        if r:
            raise msplit.MsplitError(r, "msplit_batch_graph")
        self._graph = g

    def launch(self):
        """One replay of the captured graph; returns the status like run()."""
        if self._graph is None:
            self.capture()
        return msplit.lib().msplit_graph_launch(self._graph, self.counts, self.stats,
                                                ctypes.c_void_p(self._gstream.cuda_stream))

    def close(self):
        if self._graph is not None:
            msplit.lib().msplit_graph_destroy(self._graph)
            self._graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def result(self, status):
        counts = [int(c) for c in self.counts]
        stats = [s.as_dict() for s in self.stats]
        statuses = [0 if st["missing"] == 0 else msplit.E_INCOMPLETE for st in stats] if status == 0 else \
            [status] * len(self.pairs)
        return BatchResult(self.pairs, self.caps, counts, stats, statuses, self)

    def slices(self, i):
        off = sum(self.caps[:i])
        c = int(self.counts[i])
        return slice(off, off + c)


def run_batch(pairs, certify=True, precision="fp64", simple=False):
    opts = msplit.make_options(precision=precision, certify=certify, simple=simple)
    runner = BatchRunner(pairs, opts)
    r = runner.run()
    torch.cuda.synchronize()
    return runner.result(r)
