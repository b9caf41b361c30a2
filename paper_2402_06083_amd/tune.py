"""Autotuner of the launch parameters of a batch, with a JSON cache.

The tuned knobs are the ones the splitting method leaves free (they change
the work distribution, never the set of starting points, Section 4.1):

- ``block_size``      threads per block of the persistent kernels (128, 256);
- ``seg_points``      fine level-line points per segment, walked by two
                      lanes from its two seeds (0 = the per-type default;
                      else 64 .. 1024);
- ``points_per_turn`` M, level-line points per turn (8 or 16: the paper's
                      HPC runs use 8, its hypQuick runs 16, Section 6.3.1);
- ``fp32_switch``     MIXED only: relative step at which a lane leaves FP32.

Each candidate runs the whole batch through ``msplit_batch`` (device time
from the call's own events); a candidate whose split is not proven (exact
count, every root certified with its label, disks quarter-separated, radius
<= 1e-10: ``batch.unproven``) is rejected.  The best options are cached per
(GPU architecture, list of types, precision, polynomial: q_{l,n} or the
simplified s_{l,n}) in a JSON file:
``$MSPLIT_TUNE_CACHE``, else ``~/.cache/msplit/tune.json``.  Lookups also
read the tunings shipped with the package (``tuned_<arch>.json``, written by
this module on that GPU); the user's cache takes precedence.
"""
import argparse
import itertools
import json
import os

from . import msplit

DEFAULT_SPACE = {
    "block_size": [128, 256],
    "seg_points": [0, 64, 128, 256, 512, 1024],
    "points_per_turn": [8, 16],
}
MIXED_SWITCHES = [2.0 ** -10, 2.0 ** -14, 2.0 ** -18]
TUNED_FIELDS = ("block_size", "seg_points", "points_per_turn", "fp32_switch")


def cache_path():
    p = os.environ.get("MSPLIT_TUNE_CACHE")
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "msplit", "tune.json")


def cache_key(arch, pairs, precision, simple=False):
    types = ",".join(f"{l}:{n}" for (l, n) in pairs)
    return f"{arch}|{precision}{'+simple' if simple else ''}|{types}"


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(cache, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_arch():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def candidates(precision, space=None):
    space = dict(space or DEFAULT_SPACE)
    if precision == "mixed" and "fp32_switch" not in space:
        space["fp32_switch"] = MIXED_SWITCHES
    keys = sorted(space)
    for vals in itertools.product(*(space[k] for k in keys)):
        yield dict(zip(keys, vals))


def _options(precision, certify, cand, simple=False):
    kw = {k: cand[k] for k in TUNED_FIELDS if k in cand}
    return msplit.make_options(precision=precision, certify=certify, simple=simple, **kw)


def shipped_path(arch):
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), f"tuned_{arch}.json")


def lookup(pairs, precision="fp64", path=None, arch=None, simple=False):
    """Cached options (a dict: options, ms, default_ms) or None: the given
    cache file, else the user's cache, else the tunings shipped for arch."""
    arch = arch or device_arch()
    key = cache_key(arch, pairs, precision, simple)
    if path is not None:
        return load_cache(path).get(key)
    hit = load_cache(cache_path()).get(key)
    return hit if hit is not None else load_cache(shipped_path(arch)).get(key)


def tune(pairs, precision="fp64", space=None, repeats=2, path=None, certify=True, verbose=False, simple=False):
    """Time every candidate on the batch and cache the fastest complete one.
    Returns {"best": {...}, "ms": best device ms, "default_ms": ..., "trials": [...]}."""
    import torch
    from . import batch
    arch = device_arch()
    trials = []
    best = None
    for cand in [{}] + list(candidates(precision, space)):
        opts = _options(precision, certify, cand, simple)
        try:
            runner = batch.BatchRunner(pairs, opts)
        except msplit.MsplitError as e:
            trials.append({"options": cand, "error": str(e)})
            continue
        ms = []
        ok = True
        for _ in range(repeats + 1):
            r = runner.run()
            torch.cuda.synchronize()
            sts = [s.as_dict() for s in runner.stats]
            if r != 0 or any(batch.unproven(s, certify) for s in sts):
                ok = False
                break
            ms.append(sts[0]["ms_device"])
        del runner
        if not ok:
            trials.append({"options": cand, "error": "incomplete split"})
            continue
        t = min(ms[1:]) if len(ms) > 1 else ms[0]
        trials.append({"options": cand, "ms": t})
        if verbose:
            print(f"[tune] {cand} {t:.3f} ms", flush=True)
        if cand and (best is None or t < best[1]):
            best = (cand, t)
    torch.cuda.empty_cache()
    default_ms = trials[0].get("ms")
    if best is None:
        raise RuntimeError("no candidate produced a complete split")
    # keep the defaults unless a candidate beats them
    chosen, t = best
    if default_ms is not None and default_ms <= t:
        chosen, t = {}, default_ms
    cache = load_cache(path)
    cache[cache_key(arch, pairs, precision, simple)] = {"options": chosen, "ms": t, "default_ms": default_ms}
    save_cache(cache, path)
    return {"best": chosen, "ms": t, "default_ms": default_ms, "trials": trials}


def tuned_options(pairs, precision="fp64", certify=True, path=None, simple=False):
    """msplit options for the batch: the cached tuning if present, else the
    defaults."""
    hit = None
    try:
        hit = lookup(pairs, precision, path, simple=simple)
    except Exception:
        hit = None
    cand = hit["options"] if hit else {}
    return _options(precision, certify, cand, simple), cand


# named batches for the command line
BATCHES = {
    "p1-24": [(0, n) for n in range(1, 25)],
    "p10": [(0, 10)],
    "p20": [(0, 20)],
    "p30": [(0, 30)],
    "mis22": [(l, s - l) for s in range(3, 23) for l in range(2, s)],
}


def main(argv=None):
    ap = argparse.ArgumentParser(description="tune launch parameters of named batches on this GPU")
    ap.add_argument("--out", default=None, help="cache file to update (default: the user cache)")
    ap.add_argument("--precision", nargs="+", default=["fp64", "mixed"], choices=["fp64", "mixed"])
    ap.add_argument("--simple", action="store_true",
                    help="Misiurewicz types through the simplified polynomials s_{l,n}")
    ap.add_argument("batches", nargs="+", choices=sorted(BATCHES))
    a = ap.parse_args(argv)
    for name in a.batches:
        pairs = BATCHES[name]
        best = None
        for prec in a.precision:
            space = None
            if best is not None:
                space = {k: [v] for k, v in best.items()}
                if prec == "mixed":
                    space["fp32_switch"] = MIXED_SWITCHES
            try:
                t = tune(pairs, prec, space=space or None, path=a.out, simple=a.simple)
            except RuntimeError as e:
                print(f"[tune] {name} {prec}: {e}", flush=True)
                continue
            if best is None:
                best = t["best"]
            print(f"[tune] {name} {prec}{' simple' if a.simple else ''}: {t['best']} {t['ms']:.3f} ms "
                  f"(defaults {t['default_ms']:.3f} ms)",
                  flush=True)


if __name__ == "__main__":
    main()
