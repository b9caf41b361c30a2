#!/usr/bin/env python3
"""Benchmark: certified roots per second of the level-line splitter on one GPU.

The metric is quoted on two workloads, both measured here:
- ``batch24`` (the headline ``value``): every p_n, n = 1..24, split in one
  batch -- 16 777 215 roots of degree 1 to 8 388 608 -- every returned root
  certified by the disk-arithmetic certificate (Thm proofRoots);
- ``p30``: p_30, 536 870 912 roots, the tip next to -2 in double-double.
Each runs in FP64 and in mixed FP32 -> FP64 precision.  A step is one pass
of the whole hot path over the workload: seeds, level-line walk, descents
(with the double-double route), collection, classification, certificate.
The inputs are the integers n themselves (no dataset exists for this
problem); nothing is cached between steps.  ``mis22`` (every Mis(l,n),
l + n <= 22, all 210 types in one batch) is measured next to them through
q_{l,n} and through the simplified s_{l,n} = p_{l+n-1} + p_{l-1}, and is
available as the headline with --workload.

Beside them: p_10, and p_20 in FP64 against FP32 steps then FP64.  After
the timed runs the CPU oracle splits and certifies the headline workload on
the host's cores (``cpu_baseline``), and every configuration up to order 24
is compared with the oracle's roots (``accuracy``: max |gpu - oracle| and
that distance over the local root separation).  Every timed call must prove
its root sets (exact counts, every root certified, disks quarter-separated,
radius <= 1e-10), else the run fails.

Prints one JSON line (metric, value, roofline of the dominant kernel, CPU
oracle baseline).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector peak (256 CU x 2.4 GHz x 128 FLOP/clk)
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector peak (packed FP32; this build's unpacked FP32 issues at the FP64 rate)

# algorithmic flops of one evaluation + update of order N: the orbit from
# its first iterate (p_1 = c, p_1' = 1 need no arithmetic) is N - 1 steps of
# 16 real flops (dz <- 2 z dz + 1, z <- z^2 + c); the Newton update
# z -= P/P' is 14; the log-Newton level-line update (T/P, log1p series,
# scaling by P/P') is 62.
FLOPS_ORBIT_STEP = 16
FLOPS_NEWTON_UPDATE = 14
FLOPS_WALK_UPDATE = 62

# HBM traffic of k_descend<false, false> on p_1..p_24 (FETCH_SIZE and WRITE_SIZE
# per dispatch, scaled by the counts of a 1 GiB device copy), valid for the
# kernel sources with this fingerprint (profiles/k_descend_batch24_traffic.md)
DESCEND_TRAFFIC_BYTES = 1258570537.0
DESCEND_TRAFFIC_SHA256 = "656b2dfb152bd8e0779723e92218ca4d1eaa922756fe367397a5c2f5b632409d"


def descend_traffic():
    """The measured bytes per launch when the kernel is the one measured, else None."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2402_06083_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return DESCEND_TRAFFIC_BYTES if h.hexdigest() == DESCEND_TRAFFIC_SHA256 else None


WORKLOADS = {
    "batch24": ("p_1..p_24 batched, all roots certified", [(0, n) for n in range(1, 25)]),
    "p20": ("p_20, all roots certified", [(0, 20)]),
    "p24": ("p_24, all roots certified", [(0, 24)]),
    "p30": ("p_30, all roots certified, tip next to -2 in double-double", [(0, 30)]),
    "mis22": ("all q_{l,n}, l >= 2, l + n <= 22, Mis(l,n) kept, all roots certified",
              [(l, s - l) for s in range(3, 23) for l in range(2, s)]),
}


def certified_roots(pairs, stats_list, what):
    """Roots counted as roots of P (p_n: all 2^(n-1); q_{l,n}: |Mis(l,n)|),
    a non-real root in the upper half plane standing for itself and its
    conjugate -- counted only when the type's root set is proven (Thm
    certif: exact count, every root certified with its label, disks
    quarter-separated, radius <= 1e-10); otherwise the run fails."""
    from paper_2402_06083_amd import batch
    tot = 0
    for (l, n), st in zip(pairs, stats_list):
        why = batch.unproven(st)
        if why:
            raise RuntimeError(f"{what}: the split of ({l},{n}) is not proven: {'; '.join(why)}")
        tot += st["total"]
    return tot


def kernel_flops(pairs, stats_list, simple=False):
    """Algorithmic flops of the walk and descent kernels over the whole call
    (per-type step counts times the per-evaluation cost of that type) and
    the kernels' device times (one launch each for the whole call).  The
    evaluated polynomial has order N = l + n (p_n, q_{l,n}) or l + n - 1
    (s_{l,n})."""
    desc = walk = 0.0
    for (l, n), st in zip(pairs, stats_list):
        N = l + n - (1 if simple and l >= 2 else 0)
        desc += st["steps_desc"] * (FLOPS_ORBIT_STEP * (N - 1) + FLOPS_NEWTON_UPDATE)
        desc += st["steps_fp32"] * (FLOPS_ORBIT_STEP * (N - 1) + FLOPS_NEWTON_UPDATE)
        walk += st["steps_walk"] * (FLOPS_ORBIT_STEP * (N - 1) + FLOPS_WALK_UPDATE)
    t_desc = stats_list[0]["ms_stage"]["descend"]
    t_walk = stats_list[0]["ms_stage"]["walk"]
    return desc, t_desc, walk, t_walk


def descent_flops_by_precision(pairs, stats_list, simple=False):
    """Algorithmic flops of the FP64 and of the FP32 descent steps."""
    f64 = f32 = 0.0
    for (l, n), st in zip(pairs, stats_list):
        N = l + n - (1 if simple and l >= 2 else 0)
        per = FLOPS_ORBIT_STEP * (N - 1) + FLOPS_NEWTON_UPDATE
        f64 += st["steps_desc"] * per
        f32 += st["steps_fp32"] * per
    return f64, f32


def distinct_parameters(runner):
    """Roots of the batch counted once per parameter c: a root of p_n whose
    exact period is n (a root of p_k, k | n, k < n, is already counted with
    p_k), conjugates included; for q_{l,n} every root (Mis(l,n))."""
    tot = 0
    for i, (l, n) in enumerate(runner.pairs):
        sl = runner.slices(i)
        real = runner.im[sl] == 0
        sel = runner.period[sl] == n if l == 0 else torch_ones_like(real)
        tot += int((sel & real).sum().item()) + 2 * int((sel & ~real).sum().item())
    return tot


def torch_ones_like(t):
    import torch
    return torch.ones_like(t, dtype=torch.bool)


def host_roots(runner, i):
    """Host copy of type i's roots from the last call (for the comparison
    with the oracle after the timed region)."""
    sl = runner.slices(i)
    return {k: getattr(runner, k)[sl].cpu().numpy() for k in ("re", "im", "re_lo", "im_lo", "period", "flags",
                                                               "radius")}


def run_gpu(pairs, precision, steps, warmup, launch="eager", tuned=None, basin=False, simple=False, keep=False):
    """eager: every call enqueued by msplit_batch (stage times from HIP
    events on the call's stream); graph: the call captured once as a
    hipGraph and replayed (msplit_graph_launch: total device time only).
    tuned: launch parameters from the autotuner (dict of option fields).
    keep: host copies of the p_n roots of the last call (agg["roots_of"])."""
    import torch
    from paper_2402_06083_amd import batch, msplit
    opts = msplit.make_options(precision=precision, certify=True, basin=basin, simple=simple, **(tuned or {}))
    runner = batch.BatchRunner(pairs, opts)
    mode = launch
    if mode == "graph":
        runner.capture()
    agg = _time_runner(runner, pairs, steps, warmup, mode, simple)
    agg["launch"] = mode
    if mode == "eager":
        agg["distinct"] = distinct_parameters(runner)
    if keep:
        agg["roots_of"] = {n: host_roots(runner, i) for i, (l, n) in enumerate(pairs) if l == 0}
    runner.close()
    del runner
    torch.cuda.empty_cache()
    return agg


def _time_runner(runner, pairs, steps, warmup, mode, simple=False):
    """The timed region holds the K calls (each ends with the library's one
    host synchronisation) and a byte copy of each call's counts and stats;
    they are checked and summed after it, call by call."""
    import ctypes
    import torch
    from paper_2402_06083_amd import msplit
    call = runner.launch if mode == "graph" else runner.run
    for _ in range(warmup):
        r = call()
    torch.cuda.synchronize()
    snap = lambda a: ctypes.string_at(ctypes.addressof(a), ctypes.sizeof(a))
    shots = []
    t0 = time.perf_counter()
    for _ in range(steps):
        r = call()
        shots.append((r, snap(runner.counts), snap(runner.stats)))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    agg = None
    for r, counts, stats in shots:
        if r not in (0,):
            raise RuntimeError(f"msplit_batch failed: {msplit.strerror(r)}")
        ctypes.memmove(ctypes.addressof(runner.counts), counts, len(counts))
        ctypes.memmove(ctypes.addressof(runner.stats), stats, len(stats))
        res = runner.result(r)
        sts = [st for (_, st, _) in res.per_pair]
        d, td, w, tw = kernel_flops(pairs, sts, simple)
        d64, d32 = descent_flops_by_precision(pairs, sts, simple)
        cr = certified_roots(pairs, sts, "timed call")
        if agg is None:
            agg = dict(desc=0.0, t_desc=0.0, walk=0.0, t_walk=0.0, roots=0, ms_device=0.0,
                       stages={k: 0.0 for k in msplit.Stats.STAGES})
        agg["desc"] += d
        agg["desc64"] = agg.get("desc64", 0.0) + d64
        agg["desc32"] = agg.get("desc32", 0.0) + d32
        agg["t_desc"] += td
        agg["walk"] += w
        agg["t_walk"] += tw
        agg["roots"] += cr
        agg["basin"] = agg.get("basin", 0) + sum(st.get("basin", 0) for st in sts)
        # stage times cover the whole call (every type in one launch per stage)
        agg["ms_device"] += sts[0]["ms_device"]
        for k, v in sts[0]["ms_stage"].items():
            agg["stages"][k] += v
    wall = t1 - t0
    agg["wall"] = wall
    agg["last_stats"] = sts
    return agg


def autotune(pairs, prec, other, retune=False, simple=False):
    """Launch parameters per precision: the cached tuning (the user's cache,
    else the one shipped for this GPU) or, when none is cached or retune is
    set, a tuning run now (before the timed steps)."""
    from paper_2402_06083_amd import tune
    tuned, info = {prec: None}, {}
    for p in [prec] + ([other] if other else []):
        hit = None if retune else tune.lookup(pairs, p, simple=simple)
        if hit is None:
            space = None
            if p != prec and tuned[prec] is not None:
                # the second precision keeps the tuned layout; MIXED sweeps its switch
                space = {k: [v] for k, v in tuned[prec].items()}
                if p == "mixed":
                    space["fp32_switch"] = tune.MIXED_SWITCHES
            t = tune.tune(pairs, p, space=space or None, simple=simple)
            hit = {"options": t["best"], "ms": t["ms"], "default_ms": t["default_ms"], "source": "tuned now"}
        else:
            hit = dict(hit, source="cache")
        tuned[p] = hit["options"]
        info[p] = hit
    return tuned, info


def run_streamed(n, steps=1, warmup=1):
    """p_n streamed (msplit_split_streamed) with buffers allocated once; wall
    time of the steps (one host synchronisation per chunk and partition)."""
    import torch
    from paper_2402_06083_amd import msplit
    opts = msplit.make_options(certify=True)
    b = msplit.stream_buffers(0, n, opts)
    for _ in range(warmup):
        msplit.split_streamed(0, n, opts, buffers=b, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = msplit.split_streamed(0, n, opts, buffers=b, check=False)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    st = r.stats
    from paper_2402_06083_amd import batch
    why = batch.unproven(st) if r.status == 0 else [f"status {r.status}"]
    if why:
        raise RuntimeError(f"streamed p_{n}: the split is not proven: {'; '.join(why)}")
    res = {"value": st["total"] / wall, "ms_per_step": 1e3 * wall, "status": r.status,
           "roots": st["total"], "certified_upper_half": st["certified"], "dd_routed": st["dd_routed"],
           "max_certified_radius": st["max_radius"], "min_sep": st["min_sep"],
           "stage_ms": {k: round(v, 1) for k, v in st["ms_stage"].items()},
           "workspace_bytes": b.ws_bytes}
    del r, b
    torch.cuda.empty_cache()
    return res


def work_per_root(stats_list):
    roots = sum(st["total"] for st in stats_list)
    if not roots:
        return None
    s = lambda k: sum(st[k] for st in stats_list)
    return {"lift_evaluations": s("steps_lift") / roots, "walk_evaluations": s("steps_walk") / roots,
            "descent_steps": (s("steps_desc") + s("steps_fp32")) / roots,
            "descent_steps_fp32": s("steps_fp32") / roots, "double_double_steps": s("steps_dd") / roots}


def blended_roofline(agg):
    """Descent kernels of a MIXED run: FP64 and FP32 steps each against their
    own vector peak, time-weighted (sum of flops_p / peak_p over the time),
    beside the FP64-only fraction."""
    t = agg["t_desc"] * 1e-3
    if t <= 0:
        return None
    f64, f32 = agg.get("desc64", 0.0), agg.get("desc32", 0.0)
    return {"blended_frac": (f64 / (FP64_PEAK_TFLOPS * 1e12) + f32 / (FP32_PEAK_TFLOPS * 1e12)) / t,
            "fp64_frac": f64 / (FP64_PEAK_TFLOPS * 1e12) / t,
            "fp32_share_of_flops": f32 / (f32 + f64) if f32 + f64 else 0.0}


def host_info():
    """CPU model, hardware threads and RAM of this host (for the record)."""
    model, ram = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_threads": os.cpu_count(), "ram_gib": ram}


def cpu_baseline(max_n=24):
    """The oracle as it stands on this host's cores, on the headline
    workload: p_1..p_max_n split and every root certified (long double, its
    own OpenMP threads).  Returns the record and the oracle's roots, which
    the accuracy check then compares with the GPU's."""
    import oracle
    t0 = time.perf_counter()
    roots = 0
    splits = {}
    for n in range(1, max_n + 1):
        r = oracle.split(0, n)
        ok, rad = oracle.certify(0, n, r.re_hi, r.im_hi, r.re_lo, r.im_lo, r.period)
        nr = int((r.im_hi[ok & 1 == 1] == 0).sum())
        roots += nr + 2 * (int((ok & 1).sum()) - nr)
        splits[n] = r
    dt = time.perf_counter() - t0
    rec = {"value": roots / dt, "unit": "certified roots/s", "cores": oracle.max_threads(), "kind": "oracle",
           "sample": f"the whole headline workload: p_1..p_{max_n} split and certified by the long-double "
                     f"oracle ({roots} roots, {dt:.1f} s)", **host_info()}
    return rec, splits


def error_vs_oracle(g, o):
    """Max |gpu - oracle| over a nearest-neighbour matching of the GPU roots g
    (dict of host arrays) onto the oracle's o, the max of that distance over
    the local separation of the oracle root (nearest other root or
    conjugate), and whether the sets are identical in the tested sense (same
    count, a bijection, every distance <= 1e-10 and <= a quarter of the
    separation, equal period labels and real flags)."""
    import numpy as np
    from scipy.spatial import cKDTree
    if len(g["re"]) != len(o.re_hi):
        return {"identical": False, "why": f"count {len(g['re'])} against {len(o.re_hi)}"}
    tree = cKDTree(np.stack([o.re_hi, o.im_hi], axis=1))
    d, idx = tree.query(np.stack([g["re"], g["im"]], axis=1), k=1)
    if len(o.re_hi) > 1:
        sep = tree.query(np.stack([o.re_hi, o.im_hi], axis=1), k=2)[0][:, 1]
    else:
        sep = np.full(1, np.inf)
    sep = np.minimum(sep, np.where(o.im_hi > 0, 2 * o.im_hi, np.inf))
    ratio = d / sep[idx]
    identical = (len(np.unique(idx)) == len(idx) and d.max() <= 1e-10 and ratio.max() <= 0.25
                 and np.array_equal(g["period"], o.period[idx]) and np.array_equal(g["im"] == 0, o.im_hi[idx] == 0))
    out = {"identical": bool(identical), "max_abs": float(d.max()), "max_over_sep": float(ratio.max())}
    dd = (g["flags"] & 8) != 0  # MSPLIT_R_DD: compare the double-double values
    if dd.any():
        j = idx[dd]
        ere = (g["re"][dd] - o.re_hi[j]) + (g["re_lo"][dd] - o.re_lo[j])
        eim = (g["im"][dd] - o.im_hi[j]) + (g["im_lo"][dd] - o.im_lo[j])
        out["max_abs_double_double"] = float(max(np.abs(ere).max(), np.abs(eim).max()))
    return out


def accuracy(roots_of, splits):
    """Per-workload error against the oracle: the worst type."""
    worst = {"identical": True, "max_abs": 0.0, "max_over_sep": 0.0, "types_compared": 0}
    for n, g in sorted(roots_of.items()):
        if n not in splits:
            continue
        e = error_vs_oracle(g, splits[n])
        worst["types_compared"] += 1
        if not e["identical"]:
            worst["identical"] = False
            worst.setdefault("differs", []).append(n)
        for k in ("max_abs", "max_over_sep", "max_abs_double_double"):
            if k in e:
                worst[k] = max(worst.get(k, 0.0), e[k])
    worst["max_certified_radius"] = max(float(g["radius"].max()) for g in roots_of.values())
    return worst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch24", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-compare", action="store_true", help="skip the second precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-p30", action="store_true", help="skip the period-30 measurement")
    ap.add_argument("--p30-steps", type=int, default=2)
    ap.add_argument("--no-frontier", action="store_true",
                    help="skip the streamed splits of p_31, p_32 and p_33")
    ap.add_argument("--frontier", type=int, nargs="+", default=[31, 32, 33],
                    help="orders of the streamed splits")
    ap.add_argument("--no-mis22", action="store_true",
                    help="skip the Misiurewicz batch (q_{l,n} and s_{l,n} routes)")
    ap.add_argument("--simple", action="store_true",
                    help="Misiurewicz headline workloads through the simplified s_{l,n}")
    ap.add_argument("--no-graph", action="store_true", help="skip the hipGraph replay measurement")
    ap.add_argument("--no-basin", action="store_true",
                    help="skip the measurement with the Newton-basin proof (MSPLIT_F_BASIN)")
    ap.add_argument("--no-tune", action="store_true", help="default launch parameters instead of the tuned ones")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner before the timed steps even when a tuning is cached")
    ap.add_argument("--no-small", action="store_true", help="skip the p_10 and p_20 lines")
    ap.add_argument("--small-steps", type=int, default=20)
    ap.add_argument("--cpu-max-n", type=int, default=24,
                    help="the oracle baseline splits and certifies p_1..p_N (default: the headline workload)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device copy (scale of the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not a run)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    desc, pairs = WORKLOADS[args.workload]
    main_prec = args.precision
    other = "mixed" if main_prec == "fp64" else "fp64"
    tuned = {main_prec: None, other: None}
    tune_info = {}
    if not args.no_tune:
        tuned, tune_info = autotune(pairs, main_prec, None if args.no_compare else other, args.retune,
                                    args.simple)
    res = run_gpu(pairs, main_prec, args.steps, args.warmup, "eager", tuned[main_prec], simple=args.simple,
                  keep=True)
    value = res["roots"] / res["wall"]
    ms_per_step = 1e3 * res["wall"] / args.steps
    # dominant kernel: the stage with the larger device time
    if res["t_desc"] >= res["t_walk"]:
        kname, flops, tms = "k_descend", res["desc"], res["t_desc"]
    else:
        kname, flops, tms = "k_walk", res["walk"], res["t_walk"]
    achieved = flops / (tms * 1e-3) / 1e12 if tms > 0 else 0.0
    out = {
        "metric": "certified roots/sec at period 24 batched & period 30; plain FP64 vs mixed precision",
        "value": value,
        "unit": "certified roots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32+f64",
        "data": "synthetic: the integers n themselves (no dataset exists for this problem)",
        "config": {"workload": desc, "pairs": len(pairs), "roots_per_step": res["roots"] // args.steps,
                   "precision": main_prec, "certified": True, "parallelism": "single GPU",
                   "polynomial": "s_{l,n}" if args.simple else "p_n / q_{l,n}",
                   "launch": "eager: msplit_batch per step, one host synchronisation per call",
                   "tuning": tune_info},
        "roofline": {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": descend_traffic() if (kname == "k_descend" and args.workload == "batch24"
                                                      and main_prec == "fp64") else None,
                     "traffic_unit": "bytes per launch",
                     "kernel_ms_per_step": tms / args.steps},
        "stage_ms_per_step": {k: v / args.steps for k, v in res["stages"].items()},
        # the other evaluation-bound kernel, same accounting
        "walk": {"kernel": "k_walk", "tflops": res["walk"] / (res["t_walk"] * 1e-3) / 1e12 if res["t_walk"] else 0.0,
                 "frac": res["walk"] / (res["t_walk"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS if res["t_walk"] else 0.0,
                 "evaluations_per_step": sum(st["steps_walk"] for st in res["last_stats"])},
        # the work per root that replaces the paper's W_N (level-line points
        # and descent steps per root): the instrumented counts of the last step
        "work_per_root": work_per_root(res["last_stats"]),
        "distinct_parameters": res.get("distinct"),
        # the sizes the collection kernels work on, per step: starts, the
        # candidates left by the local identification (the sort's entries),
        # the identified roots, the roots kept by the classification
        "collection_sizes": {k: sum(st[f] for st in res["last_stats"]) for k, f in
                             (("starts", "starts"), ("candidates", "sorted"), ("kept", "unique"),
                              ("discarded", "discarded"))},
    }
    if not args.no_graph:
        rg = run_gpu(pairs, main_prec, args.steps, args.warmup, "graph", tuned[main_prec], simple=args.simple)
        out["graph"] = {"value": rg["roots"] / rg["wall"], "ms_per_step": 1e3 * rg["wall"] / args.steps,
                        "device_ms_per_step": rg["ms_device"] / args.steps,
                        "launch": "whole call captured once as a hipGraph, replayed each step"}
    if not args.no_basin:
        rb = run_gpu(pairs, main_prec, args.steps, args.warmup, "eager", tuned[main_prec], basin=True,
                     simple=args.simple)
        out["basin"] = {"value": rb["roots"] / rb["wall"], "ms_per_step": 1e3 * rb["wall"] / args.steps,
                        "roots_with_basin_per_step": rb["basin"] // args.steps,
                        "what": "the same workload with a proven disk of Newton convergence around every "
                                "certified root (Thm proofContract, MSPLIT_F_BASIN)"}
    kept = {"main": res.pop("roots_of")}
    if not args.no_compare:
        r2 = run_gpu(pairs, other, args.steps, args.warmup, "eager", tuned[other], simple=args.simple, keep=True)
        kept[other] = r2.pop("roots_of")
        out[other] = {"value": r2["roots"] / r2["wall"], "ms_per_step": 1e3 * r2["wall"] / args.steps,
                      "stage_ms_per_step": {k: v / args.steps for k, v in r2["stages"].items()},
                      "descent_roofline": blended_roofline(r2)}
    # the small configurations: p_10, and p_20 in FP64 against FP32 -> FP64
    small = {}
    if not args.no_small:
        for name, n in (("p10", 10), ("p20", 20)):
            sp = [(0, n)]
            ts = {"fp64": None, "mixed": None}
            if not args.no_tune:
                ts, info = autotune(sp, "fp64", "mixed", args.retune)
                tune_info[name] = info
            small[name] = {}
            precs = ("fp64", "mixed", "dd") if n == 20 else ("fp64", "mixed")
            for prec in precs:
                # MSPLIT_DD: every descent in double-double, with the FP64 launch options
                rs = run_gpu(sp, prec, args.small_steps, args.warmup, "eager", ts["fp64" if prec == "dd" else prec],
                             keep=True)
                small[name][prec] = {"value": rs["roots"] / rs["wall"],
                                     "ms_per_step": 1e3 * rs["wall"] / args.small_steps,
                                     "device_ms_per_step": rs["ms_device"] / args.small_steps,
                                     "steps_fp32_per_root": rs["last_stats"][0]["steps_fp32"] / rs["roots"]
                                     * args.small_steps}
                kept[f"{name}_{prec}"] = rs.pop("roots_of")
        out["p10"] = {"workload": "p_10, all 512 roots certified", "unit": "certified roots/s", **small["p10"]}
        out["p20"] = {"workload": "p_20, all 524 288 roots certified: plain FP64 against FP32 steps then FP64 "
                                  "(and every descent in double-double, the DD precision)",
                      "unit": "certified roots/s", **small["p20"]}
    if not args.no_p30 and args.workload != "p30":
        p30 = {}
        p30_pairs = WORKLOADS["p30"][1]
        t30 = {main_prec: None, other: None}
        if not args.no_tune:
            t30, i30 = autotune(p30_pairs, main_prec, None if args.no_compare else other, args.retune)
            tune_info["p30"] = i30
        for prec in ([main_prec] if args.no_compare else [main_prec, other]):
            r3 = run_gpu(p30_pairs, prec, args.p30_steps, 1, "eager", t30[prec])
            st = r3["last_stats"][0]
            p30[prec] = {"value": r3["roots"] / r3["wall"], "ms_per_step": 1e3 * r3["wall"] / args.p30_steps,
                         "roots_per_step": r3["roots"] // args.p30_steps,
                         "stage_ms_per_step": {k: v / args.p30_steps for k, v in r3["stages"].items()},
                         "max_certified_radius": st["max_radius"], "min_sep": st["min_sep"],
                         "steps_fp32": st["steps_fp32"]}
            if prec == "mixed":
                p30[prec]["same_work_as_fp64"] = True
                p30[prec]["note"] = ("FP32 steps run on p_n of order <= 20 only: at order 30 the mixed "
                                     "call runs the FP64 kernels, and its rate differs from FP64 by noise")
        out["p30"] = {"workload": WORKLOADS["p30"][0], "unit": "certified roots/s",
                      "accuracy": "every root certified in a disk of radius <= max_certified_radius; "
                                  "parity with the oracle: tests/test_gpu_oracle_exact.py", **p30}
    if not args.no_mis22 and args.workload != "mis22":
        m22 = {}
        m_pairs = WORKLOADS["mis22"][1]
        for route, simple in (("q", False), ("s", True)):
            tm = {main_prec: None}
            if not args.no_tune:
                tm, im = autotune(m_pairs, main_prec, None, args.retune, simple)
                tune_info["mis22_" + route] = im
            rm = run_gpu(m_pairs, main_prec, args.steps, args.warmup, "eager", tm[main_prec], simple=simple)
            m22[route] = {"value": rm["roots"] / rm["wall"], "ms_per_step": 1e3 * rm["wall"] / args.steps,
                          "roots_per_step": rm["roots"] // args.steps,
                          "stage_ms_per_step": {k: v / args.steps for k, v in rm["stages"].items()}}
        m22["s"]["speedup_vs_q"] = m22["q"]["ms_per_step"] / m22["s"]["ms_per_step"]
        out["mis22"] = {"workload": WORKLOADS["mis22"][0], "unit": "certified roots/s",
                        "q": dict(m22["q"], polynomial="q_{l,n} = p_{l+n} - p_l"),
                        "s": dict(m22["s"], polynomial="s_{l,n} = p_{l+n-1} + p_{l-1} (eq. polySimple)")}
    if not args.no_frontier:
        out["frontier"] = {"unit": "certified roots/s", "workload": "p_n split chunk by chunk "
                           "(msplit_split_streamed, chunks of 2^28 starts), every root certified",
                           **{f"p{n}": run_streamed(n) for n in args.frontier}}
    if args.copy_probe:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 1 << 30
    if not args.no_cpu_baseline:
        out["cpu_baseline"], splits = cpu_baseline(args.cpu_max_n)
        # error against the oracle, per configuration (the worst type)
        acc = {}
        if args.workload == "batch24":
            acc["batch24_" + main_prec] = accuracy(kept["main"], splits)
            if other in kept:
                acc["batch24_" + other] = accuracy(kept[other], splits)
        for name, n in (("p10", 10), ("p20", 20)):
            for prec in ("fp64", "mixed", "dd"):
                if f"{name}_{prec}" in kept:
                    acc[f"{name}_{prec}"] = accuracy(kept[f"{name}_{prec}"], splits)
        out["accuracy"] = {"what": "max |gpu - oracle| and max |gpu - oracle| / local separation over a "
                                   "nearest-neighbour matching with the oracle's roots (long double, "
                                   "double-double polish), per configuration; identical = same count, a "
                                   "bijection within 1e-10 and a quarter of the separation, equal period "
                                   "labels and real flags", **acc}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
