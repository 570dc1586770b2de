"""Autotuner for the sigma kernels' launch shapes, single-space and batched.

Knobs (libsqd tuning keys, 0 = the library's automatic choice):
  same-spin   rows staged per workgroup (1, 2, 4, 8) x waves per workgroup (4, 8, 16)
  alpha-beta  grouped kernel: alpha singles per unit (1, 2, 4, 8) x waves (4, 8, 16);
              row-staged kernel: sources per pass (1, 2, 4, 8) x waves;
              kernel grouped by source string: waves

Tile choices interact through the caches (the alpha-beta intermediate streams
through the same L2 and Infinity Cache the same-spin tables live in), so every
candidate is timed on the whole product, not on one term: a coordinate search
tunes the same-spin knobs with the alpha-beta ones automatic, then the
alpha-beta knobs with the best same-spin setting applied.  Times are HIP events
on the context's stream.

``tune`` tunes one space's sigma; ``tune_batched`` tunes the persistent
batched solver for a list of spaces by timing short batched solves (a fixed
number of iterations, no convergence test) and applies the same knobs, which
the batched launch reads.  Results are cached in a JSON file keyed by the
device and a signature of the space (or of the batch), so a workload is tuned
once per machine.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Sequence, Tuple

from . import sqd

CACHE = os.environ.get("SQD_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json"))

Setting = Tuple[int, ...]   # key, value, key, value, ...

# rows staged x waves (whole rows), or windows of source strings (for rows too
# long to stage several whole)
SS_KNOBS: List[Setting] = ([(sqd.TUNE_SS_WINDOW, 1, sqd.TUNE_SS_ROWS, r, sqd.TUNE_SS_WAVES, w)
                            for r in (1, 2, 4, 8) for w in (4, 8, 16)]
                           + [(sqd.TUNE_SS_WINDOW, 2, sqd.TUNE_SS_ROWS, 0, sqd.TUNE_SS_WAVES, 0)])
AB_KNOBS: List[Setting] = (
    [(sqd.TUNE_AB_VARIANT, 1, sqd.TUNE_AB_GROUP, g, sqd.TUNE_AB_WAVES, w) for g in (1, 2, 4, 8) for w in (4, 8, 16)]
    + [(sqd.TUNE_AB_VARIANT, 2, sqd.TUNE_AB_CHUNK, k, sqd.TUNE_AB_WAVES, w) for k in (1, 2, 4, 8) for w in (8, 16)]
    + [(sqd.TUNE_AB_VARIANT, 3, sqd.TUNE_AB_WAVES, w) for w in (8, 16)])
# the batched solver has no row-staged alpha-beta variant
AB_KNOBS_BATCHED: List[Setting] = [s for s in AB_KNOBS if s[1] == 1]
ALL_KEYS = (sqd.TUNE_SS_ROWS, sqd.TUNE_SS_WAVES, sqd.TUNE_AB_VARIANT, sqd.TUNE_AB_GROUP, sqd.TUNE_AB_CHUNK,
            sqd.TUNE_AB_WAVES, sqd.TUNE_SS_WINDOW)


def signature(space: "sqd.Space", precision: int) -> str:
    i = space.info()
    return (f"na{i['na']}_nb{i['nb']}_norb{i['norb']}_e{i['nalpha']}-{i['nbeta']}"
            f"_s{i['nnz_single'][0]}-{i['nnz_single'][1]}_d{i['nnz_double'][0]}-{i['nnz_double'][1]}_p{precision}")


def batch_signature(spaces: Sequence["sqd.Space"], mode: int) -> str:
    import hashlib
    h = hashlib.sha256("|".join(signature(s, 0) for s in spaces).encode()).hexdigest()[:16]
    return f"batch{len(spaces)}_{h}_m{mode}"


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) + ":" + str(torch.cuda.get_device_properties(0).gcnArchName)


def _load() -> Dict:
    if os.path.exists(CACHE):
        try:
            return json.load(open(CACHE))
        except (OSError, ValueError):
            return {}
    return {}


def _store(key: str, value) -> None:
    cache = _load()
    cache[key] = value
    try:
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass


def _apply(ctx, setting: Setting) -> None:
    for k, v in zip(setting[0::2], setting[1::2]):
        ctx.set_tuning(k, v)


def reset(ctx) -> None:
    """Restore every sigma launch knob to the library's automatic choice."""
    for k in ALL_KEYS:
        ctx.set_tuning(k, 0)


def _search(ctx, groups, measure, log) -> Dict:
    """Coordinate search: for each knob group in turn, keep the fastest
    setting (later groups are timed with the earlier winners applied)."""
    result = {}
    for name, knobs in groups:
        best = None
        for setting in knobs:
            try:
                _apply(ctx, setting)
                ms = measure()
            except sqd.SQDError:
                continue
            finally:
                for k in setting[0::2]:
                    ctx.set_tuning(k, 0)
            if log:
                log(f"tune {name} {setting}: {ms:.4f} ms")
            if best is None or ms < best[1]:
                best = (list(setting), ms)
        if best is None:
            raise RuntimeError(f"no valid setting for {name}")
        _apply(ctx, best[0])
        result[name] = best
    return result


def tune(space: "sqd.Space", precision: int = sqd.FP64, reps: int = 10, use_cache: bool = True,
         log=None) -> Dict:
    """Tune the context of ``space`` for its full sigma product; returns
    {group: (setting, ms)} and leaves the fastest setting applied."""
    import torch
    ctx = space.ctx
    key = _device_name() + "|" + signature(space, precision)
    if use_cache:
        cached = _load().get(key)
        if cached:
            reset(ctx)
            for name in ("ss", "ab"):
                _apply(ctx, cached[name][0])
            return cached
    c = torch.randn(space.dim, dtype=torch.float64, device=f"cuda:{ctx.device}")
    out = torch.empty_like(c)
    stream = ctx.stream

    def measure():
        for _ in range(2):
            space.sigma(c, out, precision=precision)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            space.sigma(c, out, precision=precision)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    reset(ctx)
    result = _search(ctx, (("ss", SS_KNOBS), ("ab", AB_KNOBS)), measure, log)
    if use_cache:
        _store(key, result)
    return result


def tune_batched(ctx, spaces: Sequence["sqd.Space"], mode: int = sqd.DAV_MIXED, iterations: int = 10,
                 use_cache: bool = True, log=None) -> Dict:
    """Tune the batched solver's tiles for ``spaces``: each candidate runs
    ``iterations`` batched Davidson iterations (tolerance 1e-300, so no space
    stops early) and the wall time after the first is compared.  Leaves the
    fastest setting applied on ``ctx``."""
    import torch
    key = _device_name() + "|" + batch_signature(spaces, mode)
    if use_cache:
        cached = _load().get(key)
        if cached:
            reset(ctx)
            for name in ("ss", "ab"):
                _apply(ctx, cached[name][0])
            return cached

    def run(n):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.davidson_batched(spaces, tol=1e-300, max_iter=n, mode=mode)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    def measure():
        # difference of two lengths removes the plan and graph set-up
        return 1e3 * (run(iterations + 2) - run(2)) / iterations

    reset(ctx)
    result = _search(ctx, (("ss", SS_KNOBS), ("ab", AB_KNOBS_BATCHED)), measure, log)
    if use_cache:
        _store(key, result)
    return result
