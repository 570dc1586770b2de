"""Autotuner for the sigma kernels' launch shapes and paths.

For one space it times every allowed setting of each tuning knob of libsqd
(rows staged per same-spin workgroup, waves per workgroup, the direct
alpha-beta variant and its chunking, the alpha-beta algorithm) with HIP events
on the context's stream, one term at a time, and keeps the fastest.  Results
are cached in a JSON file keyed by the device name and a signature of the
space (strings per spin, orbitals, electrons, table sizes), so a workload is
tuned once per machine.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

from . import sqd

CACHE = os.environ.get("SQD_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json"))

# knob -> candidate values (0 = the library's automatic choice)
KNOBS = {
    "ss": [(sqd.TUNE_SS_ROWS, r, sqd.TUNE_SS_WAVES, w) for r in (0, 1, 2, 4, 8) for w in (4, 8, 16)],
    "ab": ([(sqd.TUNE_AB_VARIANT, 1, sqd.TUNE_AB_WAVES, w) for w in (4, 8, 16)]
           + [(sqd.TUNE_AB_VARIANT, 2, sqd.TUNE_AB_CHUNK, k) for k in (1, 2, 4, 8)]),
}


def signature(space: "sqd.Space", precision: int) -> str:
    i = space.info()
    return (f"na{i['na']}_nb{i['nb']}_norb{i['norb']}_e{i['nalpha']}-{i['nbeta']}"
            f"_s{i['nnz_single'][0]}-{i['nnz_single'][1]}_d{i['nnz_double'][0]}-{i['nnz_double'][1]}_p{precision}")


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) + ":" + str(torch.cuda.get_device_properties(0).gcnArchName)


def _time(space, c, out, precision, terms, reps):
    import torch
    stream = space.ctx.stream
    space.sigma(c, out, precision=precision, terms=terms)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        space.sigma(c, out, precision=precision, terms=terms)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def _load() -> Dict:
    if os.path.exists(CACHE):
        try:
            return json.load(open(CACHE))
        except (OSError, ValueError):
            return {}
    return {}


def _apply(ctx, setting):
    for k, v in zip(setting[0::2], setting[1::2]):
        ctx.set_tuning(k, v)


def tune(space: "sqd.Space", precision: int = sqd.FP64, reps: int = 5, use_cache: bool = True,
         log=None) -> Dict:
    """Tune the context of ``space`` for it; returns {knob: (setting, ms)} and
    leaves the fastest setting applied."""
    import torch
    ctx = space.ctx
    key = _device_name() + "|" + signature(space, precision)
    cache = _load() if use_cache else {}
    if key in cache:
        best = cache[key]
        for name in ("ss", "ab"):
            _apply(ctx, best[name][0])
        return best
    c = torch.randn(space.dim, dtype=torch.float64, device=f"cuda:{ctx.device}")
    out = torch.empty_like(c)
    result = {}
    for name, terms in (("ss", sqd.TERM_BB), ("ab", sqd.TERM_AB)):
        best = None
        for setting in KNOBS[name]:
            try:
                _apply(ctx, setting)
                ms = _time(space, c, out, precision, terms, reps)
            except sqd.SQDError:
                continue
            if log:
                log(f"tune {name} {setting}: {ms:.4f} ms")
            if best is None or ms < best[1]:
                best = (list(setting), ms)
        if best is None:
            raise RuntimeError(f"no valid setting for {name}")
        _apply(ctx, best[0])
        result[name] = best
    if use_cache:
        cache = _load()
        cache[key] = result
        try:
            with open(CACHE, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return result
