#!/usr/bin/env python3
"""Benchmark of the SQD hot path on one MI355X.

A step is one full sigma = H c (diagonal, alpha-alpha, beta-beta and
alpha-beta terms, FP64) over the 4.0e6-determinant workload (norb 16, 8+8
electrons, 2000 HF-biased strings per spin, seeded synthetic integrals).
``value`` is determinants per second per sigma (Gdet/s) with all inputs
resident in HBM.  The same run also reports:

  * FP32-sigma throughput (off-diagonal terms in FP32, diagonal in FP64);
  * Davidson time-to-converge for the lowest root, FP64 vs FP32-sigma + FP64
    refinement, both from the same start vector and to the same residual
    tolerance, with the energy difference to the stored oracle value;
  * the roofline of the dominant kernel, timed live with HIP events on the
    stream it runs on;
  * the CPU oracle timed on a bounded sample of rows on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg2]
       python bench.py --leg kh|rdm|roots [--workload cfg2|cfg3|cfg5|full14]   (secondary legs)
       python bench.py --leg batched [--tune]   (64 uneven spaces: batched vs one by one)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
COPY_BYTES = 1 << 28
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--no-davidson", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--profile-only", action="store_true",
                    help="only the timed sigma loop (for profilers)")
    ap.add_argument("--leg", choices=("kh", "rdm", "roots", "batched"), default=None,
                    help="instead of the headline: time the Knowles-Handy alpha-beta path against the direct one, "
                         "the RDM backward kernels, the four lowest roots, or the batched solver on 64 uneven "
                         "spaces against solving them one by one (one JSON line each)")
    ap.add_argument("--tune", action="store_true",
                    help="batched leg: also time after tuning the batched tiles for these spaces")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "libsqd runs on one GPU; --gpus must be 1 "
                          "(the multi-GPU sharding is designed but not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2601_16169_amd import inputs as I
    from paper_2601_16169_amd import sqd

    assert torch.cuda.is_available(), "bench needs a HIP device"
    dev = "cuda:0"
    if a.leg == "batched":
        _leg_batched(a)
        return
    prob = I.WORKLOADS[a.workload]()
    log(f"workload {prob.name}: dim {prob.dim}")
    stream = torch.cuda.current_stream(0)
    ctx = sqd.Context(0, stream)
    ctx.set_hamiltonian(prob.ints.h, prob.ints.eri, prob.ints.ecore)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sp = ctx.build_space(prob.nalpha, prob.nbeta, prob.astr, prob.bstr)
    torch.cuda.synchronize()
    t_tables = time.perf_counter() - t0
    info = sp.info()
    log(f"tables built in {t_tables:.3f} s: {info}")
    c = torch.tensor(I.random_vector(sp.dim, 21), device=dev)
    out = torch.empty_like(c)
    if a.leg:
        _leg(a, ctx, sp, prob, c, out, info)
        return

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    # ---- headline: FP64 sigma, all terms
    t64 = timed(lambda: sp.sigma(c, out, precision=sqd.FP64), a.steps, a.warmup)
    log(f"sigma fp64 {t64 * 1e3:.3f} ms")
    if a.profile_only:
        # plain copy of known size, for scaling the HBM byte counters
        src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {COPY_BYTES} bytes read + written per copy")
        return
    t32 = timed(lambda: sp.sigma(c, out, precision=sqd.FP32), a.steps, a.warmup)
    log(f"sigma fp32 {t32 * 1e3:.3f} ms")

    # ---- per-term times (HIP events on the context's stream)
    def event_time(fn, reps):
        fn()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / 1e3 / reps

    terms = {}
    for name, mask in (("diag", sqd.TERM_DIAG), ("aa", sqd.TERM_AA), ("bb", sqd.TERM_BB), ("ab", sqd.TERM_AB)):
        terms[name] = {
            "fp64_ms": 1e3 * event_time(lambda: sp.sigma(c, out, precision=sqd.FP64, terms=mask), a.steps),
            "fp32_ms": 1e3 * event_time(lambda: sp.sigma(c, out, precision=sqd.FP32, terms=mask), a.steps),
        }
    log(f"terms {terms}")

    # ---- per-kernel times: HIP events recorded by the library on its stream
    ctx.profile(True)
    for _ in range(a.steps):
        sp.sigma(c, out, precision=sqd.FP64)
    kern = ctx.profile_report()
    ctx.profile(False)
    kernels = {k: {"calls_per_step": n / a.steps, "ms_per_step": ms / a.steps, "ms_per_launch": ms / n}
               for k, (n, ms) in kern.items()}
    log(f"kernels {kernels}")
    roofline = _roofline(kernels, info, sp, prob)
    conn = info["conn_per_sigma"]
    result = {
        "metric": "sigma (H.c) Gdet/s + Davidson time-to-converge, mixed vs FP64, one GPU",
        "value": sp.dim / t64 / 1e9,
        "unit": "Gdet/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": t64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded integrals and HF-biased strings; the paper's molecules are not available)",
        "config": {"workload": prob.name, "norb": prob.norb, "nalpha": prob.nalpha, "nbeta": prob.nbeta,
                   "strings_per_spin": [int(sp.na), int(sp.nb)], "dim": int(sp.dim),
                   "connections_per_sigma": int(conn)},
        "sigma_fp32": {"value": sp.dim / t32 / 1e9, "unit": "Gdet/s", "ms": t32 * 1e3},
        "gconn_per_s": {"fp64": conn / t64 / 1e9, "fp32": conn / t32 / 1e9},
        "terms_ms": terms,
        "kernels": kernels,
        "tables_s": t_tables,
        "roofline": roofline,
    }

    # ---- Davidson, FP64 vs mixed
    if not a.no_davidson:
        noise = torch.tensor(I.guess_noise(sp.dim), device=dev)
        gold_path = os.path.join(ROOT, "tests", "golden", f"{a.workload}_oracle.json")
        gold = json.load(open(gold_path)) if os.path.exists(gold_path) else None
        dav = {}
        sp.davidson(tol=1e-8, noise=noise, max_iter=5)  # warm-up of every kernel
        for mode, name in ((sqd.DAV_FP64, "fp64"), (sqd.DAV_MIXED, "mixed")):
            torch.cuda.synchronize()
            t = time.perf_counter()
            E, x, rep = sp.davidson(tol=1e-8, mode=mode, switch_tol=1e-4, noise=noise)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            d = {"seconds": el, "energy": E, "iterations": rep["iterations"],
                 "iterations_fp32": rep["iterations_fp32"], "switch_iter": rep["switch_iter"],
                 "converged": rep["converged"], "residual": rep["residual"]}
            if gold:
                d["abs_err_vs_oracle_Ha"] = abs(E - gold["energy"])
            dav[name] = (d, x.clone())
            log(f"davidson {name}: {d}")
        d64, x64 = dav["fp64"]
        dmx, xmx = dav["mixed"]
        dmx["abs_err_vs_fp64_Ha"] = abs(dmx["energy"] - d64["energy"])
        dmx["vector_err_vs_fp64"] = float(1.0 - abs(torch.dot(x64, xmx)))
        result["davidson"] = {"tol": 1e-8, "fp64": d64, "mixed": dmx,
                              "speedup_mixed_vs_fp64": d64["seconds"] / dmx["seconds"],
                              "oracle_energy": gold["energy"] if gold else None}

    # ---- CPU oracle on a bounded sample of rows
    if not a.no_cpu_baseline:
        from oracle import core
        osp = core.Space.from_problem(prob)
        cnp = c.cpu().numpy()
        rng = np.random.default_rng(0)
        rows = rng.choice(sp.dim, size=min(4096, sp.dim), replace=False)
        t = time.perf_counter()
        osp.sigma_rows(cnp, rows)
        t_small = time.perf_counter() - t
        nrows = int(min(sp.dim, max(4096, len(rows) * a.cpu_seconds / max(t_small, 1e-3))))
        rows = rng.choice(sp.dim, size=nrows, replace=False)
        t = time.perf_counter()
        ref = osp.sigma_rows(cnp, rows)
        t_cpu = time.perf_counter() - t
        got = out  # last product was a term-only call: recompute the full one
        sp.sigma(c, out, precision=sqd.FP64)
        err = float(np.abs(out.cpu().numpy()[rows] - ref).max() / np.abs(ref).max())
        result["cpu_baseline"] = {"value": nrows / t_cpu / 1e9, "unit": "Gdet/s", "cores": core.num_threads(),
                                  "kind": "oracle",
                                  "sample": f"{nrows} random rows of sigma (of {sp.dim}), {t_cpu:.1f} s",
                                  "cpu_model": _cpu_model(), "gpu_vs_cpu": (sp.dim / t64) / (nrows / t_cpu),
                                  "max_rel_err_gpu_vs_oracle_rows": err}
        log(f"cpu baseline {result['cpu_baseline']}")

    print(json.dumps(result))


def _leg(a, ctx, sp, prob, c, out, info):
    """Secondary measurements, one JSON line each (not the headline)."""
    import torch
    from paper_2601_16169_amd import inputs as I
    from paper_2601_16169_amd import sqd

    def kernels(fn):
        for _ in range(a.warmup):
            fn()
        ctx.synchronize()
        ctx.profile(True)
        for _ in range(a.steps):
            fn()
        r = ctx.profile_report()
        ctx.profile(False)
        return {k: ms / n for k, (n, ms) in r.items()}

    if a.leg == "kh":
        # dense-K equivalent of the KH form: 2 x nb x norb^2 x (alpha singles);
        # the GEMM the kernel runs has K = the pair columns active in each
        # 64-target beta tile: 2 x kh_columns x (alpha singles)
        dense = 2.0 * info["nb"] * prob.norb ** 2 * info["nnz_single"][0]
        for prec, name, peak in ((sqd.FP64, "fp64", PEAK_FP64_TFLOPS), (sqd.FP32, "fp32", PEAK_FP32_TFLOPS)):
            d = kernels(lambda: sp.sigma(c, out, precision=prec, terms=sqd.TERM_AB))
            try:
                k = kernels(lambda: sp.sigma(c, out, precision=prec, terms=sqd.TERM_AB, ab_path=sqd.AB_KH))
            except sqd.SQDError as e:   # e.g. a source row too long for the KH tile's LDS
                print(json.dumps({"leg": "kh", "workload": prob.name, "precision": name, "direct_ms": d,
                                  "kh_error": str(e)}), flush=True)
                continue
            t = [v for n_, v in k.items() if n_.startswith("k_ab_kh")][0] / 1e3
            flops = 2.0 * sp.info()["kh_columns"] * info["nnz_single"][0]
            print(json.dumps({"leg": "kh", "workload": prob.name, "precision": name, "direct_ms": d, "kh_ms": k,
                              "kh_gemm_flops": flops, "kh_dense_k_flops": dense, "kh_tflops": flops / t / 1e12,
                              "kh_frac_of_mfma_peak": flops / t / 1e12 / peak}), flush=True)
    elif a.leg == "rdm":
        noise = torch.tensor(I.guess_noise(sp.dim), device="cuda:0")
        E, x, rep = sp.davidson(tol=1e-8, noise=noise)
        for two in (False, True):
            sp.rdm(x, two_body=two)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(a.steps):
                sp.rdm(x, two_body=two)
            torch.cuda.synchronize()
            print(json.dumps({"leg": "rdm", "workload": prob.name, "two_body": two,
                              "ms": (time.perf_counter() - t) / a.steps * 1e3, "energy": E}), flush=True)
    elif a.leg == "roots":
        noise = torch.tensor(I.guess_noise(sp.dim), device="cuda:0")
        for mode, name in ((sqd.DAV_FP64, "fp64"), (sqd.DAV_MIXED, "mixed")):
            torch.cuda.synchronize()
            t = time.perf_counter()
            E, X, reps = sp.davidson_roots(4, tol=1e-8, mode=mode, noise=noise, max_iter=400)
            torch.cuda.synchronize()
            print(json.dumps({"leg": "roots", "workload": prob.name, "mode": name,
                              "seconds": time.perf_counter() - t, "energies": E,
                              "iterations": [r["iterations"] for r in reps],
                              "converged": all(r["converged"] for r in reps)}), flush=True)


def _leg_batched(a):
    """64 independent spaces (norb 24, 8+8 electrons, 200-3000 strings per
    spin, shared integrals): one batched solve per mode against the
    single-space solver run on each space in turn, same tolerance."""
    import numpy as np
    import torch
    from paper_2601_16169_amd import autotune
    from paper_2601_16169_amd import inputs as I
    from paper_2601_16169_amd import sqd

    probs = I.cfg4()
    ctx = sqd.Context(0)
    ctx.set_hamiltonian(probs[0].ints.h, probs[0].ints.eri, probs[0].ints.ecore)
    torch.cuda.synchronize()
    t = time.perf_counter()
    spaces = [ctx.build_space(p.nalpha, p.nbeta, p.astr, p.bstr) for p in probs]
    torch.cuda.synchronize()
    t_tables = time.perf_counter() - t
    dims = [s.dim for s in spaces]
    conn = sum(s.info()["conn_per_sigma"] for s in spaces)
    head = {"leg": "batched", "workload": "cfg4_64_spaces_norb24_n8", "nspaces": len(spaces),
            "sum_dim": int(sum(dims)), "min_dim": int(min(dims)), "max_dim": int(max(dims)),
            "connections_per_sweep": int(conn), "tables_s": t_tables, "tol": 1e-8}

    def solve_batched(mode):
        torch.cuda.synchronize()
        t = time.perf_counter()
        E, vecs, reps, rc = ctx.davidson_batched(spaces, tol=1e-8, max_iter=600, mode=mode)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        it = [r["iterations"] for r in reps]
        del vecs
        return el, np.array(E), {"iterations_min": min(it), "iterations_max": max(it),
                                 "all_converged": all(r["converged"] for r in reps)}

    def solve_each(mode):
        torch.cuda.synchronize()
        t = time.perf_counter()
        Es = []
        for s in spaces:
            e, x, r = s.davidson(tol=1e-8, max_iter=600, mode=mode)
            Es.append(e)
            del x
        torch.cuda.synchronize()
        return time.perf_counter() - t, np.array(Es)

    ctx.davidson_batched(spaces, tol=1e-8, max_iter=3)   # warm-up of every kernel
    spaces[0].davidson(tol=1e-8, max_iter=3)
    res = dict(head)
    energies = {}
    for mode, name in ((sqd.DAV_FP64, "fp64"), (sqd.DAV_MIXED, "mixed")):
        el, E, st = solve_batched(mode)
        res[f"batched_{name}_s"] = el
        res[f"batched_{name}"] = st
        energies[f"batched_{name}"] = E
        log(f"batched {name}: {el:.3f} s {st}")
        el, E = solve_each(mode)
        res[f"one_by_one_{name}_s"] = el
        energies[f"one_by_one_{name}"] = E
        log(f"one by one {name}: {el:.3f} s")
    if a.tune:
        t = time.perf_counter()
        autotune.tune_batched(ctx, spaces, mode=sqd.DAV_MIXED, use_cache=False)
        res["tune_s"] = time.perf_counter() - t
        for mode, name in ((sqd.DAV_FP64, "fp64"), (sqd.DAV_MIXED, "mixed")):
            el, E, st = solve_batched(mode)
            res[f"tuned_batched_{name}_s"] = el
            energies[f"tuned_batched_{name}"] = E
        res["tuned_setting"] = {k: ctx.get_tuning(k) for k in autotune.ALL_KEYS}
    ref = energies["one_by_one_fp64"]
    res["max_abs_dE_vs_one_by_one_fp64_Ha"] = {k: float(np.abs(v - ref).max()) for k, v in energies.items()
                                              if k != "one_by_one_fp64"}
    res["speedup_batched_mixed_vs_one_by_one_fp64"] = res["one_by_one_fp64_s"] / res["batched_mixed_s"]
    for s in spaces:
        s.close()
    print(json.dumps(res), flush=True)


def _algorithmic(name, info, sp):
    """(bound, work per launch, unit) of one kernel, from the table counts.

    Pair-gather kernels: one multiply-add (2 flops) per Hamiltonian connection
    they evaluate.  alpha-beta: every (alpha single, beta single) pair.
    same-spin (called once per spin, the beta call also applying the
    diagonal): the singles and doubles of that spin times the strings of the
    other.  Gather, transpose: bytes read + written once.
    """
    es = 8 if "double" in name else 4
    t = info["conn_terms"]  # diag, aa, bb, ab connections per sigma
    if name.startswith(("k_ab_grouped", "k_ab_direct", "k_ab_kh")):
        return "alu", 2.0 * t[3], "flop"
    if name.startswith("k_same_spin"):
        # [aa]: alpha-alpha launch (on C^T), [bb]: beta-beta launch
        return "alu", 2.0 * (t[1] if name.endswith("[aa]") else t[2]), "flop"
    if name.startswith("k_ab_gather"):
        return "hbm", float(es) * (info["nnz_single"][0] * sp.nb + 2 * sp.dim), "byte"
    if name.startswith("k_transpose"):
        return "hbm", 2.0 * es * sp.dim, "byte"
    return None, None, None


def _traffic(name):
    """HBM bytes per launch from the committed --pmc summary of this kernel,
    or None when none is there or the kernel source changed since."""
    import hashlib
    base = name.split("<")[0]
    path = os.path.join(PROFILES, f"traffic_{base}_cfg2.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    src = vals.get("source")
    if not src or "bytes_per_launch" not in vals:
        return None
    h = hashlib.sha256()
    for f in src.split():
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest()[:16] != vals.get("source_sha256"):
        return None
    return float(vals["bytes_per_launch"])


def _lds_util(name, column=3):
    """LDS busy fraction (rocprofv3 LdsUtil; column 5: VALUBusy) of this
    kernel from the committed summary, or None when absent or the kernel
    source changed since."""
    import hashlib
    import re
    path = os.path.join(PROFILES, "lds_sigma_cfg2.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source: `([^`]*)`", text)
    h = re.search(r"source_sha256: `([0-9a-f]+)`", text)
    if not m or not h:
        return None
    d = hashlib.sha256()
    for f in m.group(1).split():
        d.update(open(os.path.join(ROOT, f), "rb").read())
    if d.hexdigest()[:16] != h.group(1):
        return None
    base, es = name.split("<")[0], ("double" if "double" in name else "float")
    for line in text.splitlines():
        cells = [c.strip() for c in line.split("|")]
        if len(cells) > column + 1 and cells[1].startswith(f"`void {base}<{es}"):
            try:
                return float(cells[column]) / 100.0
            except ValueError:
                return None
    return None


def _roofline(kernels, info, sp, prob):
    """Roofline of the kernel with the largest share of the step."""
    name = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    bound, work, unit = _algorithmic(name, info, sp)
    t = kernels[name]["ms_per_launch"] / 1e3
    if bound == "hbm":
        ach, peak, u = work / t / 1e9, PEAK_HBM_GBS, "GB/s"
    else:
        peak = PEAK_FP64_TFLOPS if "double" in name else PEAK_FP32_TFLOPS
        ach, u = work / t / 1e12, "TFLOP/s"
    return {"kernel": name, "bound": bound, "achieved": ach, "peak": peak, "unit": u, "frac": ach / peak,
            "traffic": _traffic(name), "lds_util": _lds_util(name), "valu_busy": _lds_util(name, 5),
            "algorithmic_per_launch": work, "algorithmic_unit": unit,
            "launch_ms": t * 1e3, "share_of_step": kernels[name]["ms_per_step"] / sum(
                v["ms_per_step"] for v in kernels.values())}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
