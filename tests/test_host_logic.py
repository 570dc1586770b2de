"""Host-side logic that needs no GPU: the benchmark's argument contract and its
readers of the committed counter summaries, its work accounting, and the
autotuner's search and cache."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_bench_counter_summaries_are_read_while_sources_match():
    import bench
    t = bench._traffic("k_ab_grouped<double>")
    if t is None:
        pytest.skip("sigma sources changed since the committed counter summaries were taken")
    assert 1e8 < t < 1e11
    assert 0.0 < bench._lds_util("k_ab_grouped<double>") <= 1.0
    assert 0.0 < bench._lds_util("k_ab_grouped<double>", 5) <= 1.0
    # kernels without a summary
    assert bench._traffic("k_not_a_kernel<double>") is None
    assert bench._lds_util("k_residual<24>") is None


def test_bench_traffic_is_null_once_a_source_changes(tmp_path, monkeypatch):
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "k.hip"
    src.write_text("original")
    import hashlib
    h = hashlib.sha256(b"original").hexdigest()[:16]
    (prof / "traffic_k_demo_cfg2.md").write_text(
        f"- source: `k.hip`\n- source_sha256: `{h}`\n- bytes_per_launch: `1234`\n")
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench._traffic("k_demo<double>") == 1234.0
    src.write_text("edited")
    assert bench._traffic("k_demo<double>") is None


def test_bench_algorithmic_work():
    import bench

    class Sp:
        nb = 10
        dim = 100
    info = {"conn_terms": [100, 7, 9, 40], "nnz_single": [3, 4]}
    assert bench._algorithmic("k_ab_grouped<double>", info, Sp) == ("alu", 80.0, "flop")
    assert bench._algorithmic("k_same_spin<double>[aa]", info, Sp) == ("alu", 14.0, "flop")
    assert bench._algorithmic("k_same_spin<float>[bb]", info, Sp) == ("alu", 18.0, "flop")
    # gather: Y rows (alpha singles x nb) read once, sigma read and written
    assert bench._algorithmic("k_ab_gather<double>", info, Sp) == ("hbm", 8.0 * (3 * 10 + 200), "byte")
    assert bench._algorithmic("k_transpose<float>", info, Sp) == ("hbm", 800.0, "byte")
    assert bench._algorithmic("k_other", info, Sp) == (None, None, None)


class FakeCtx:
    """Records tuning calls; rejects one setting like the library would."""

    def __init__(self):
        self.tune = {}

    def set_tuning(self, key, value):
        from paper_2601_16169_amd import sqd
        if key == sqd.TUNE_SS_ROWS and value == 8:
            raise sqd.SQDError(-9, "does not fit")
        self.tune[key] = value


def test_autotune_search_keeps_the_fastest_valid_setting():
    from paper_2601_16169_amd import autotune, sqd
    ctx = FakeCtx()
    # time = rows + waves / 100 (smallest rows first), except rows 2 which is fastest
    def measure():
        r, w = ctx.tune.get(sqd.TUNE_SS_ROWS, 0), ctx.tune.get(sqd.TUNE_SS_WAVES, 0)
        return (0.5 if r == 2 else float(r)) + w / 100.0
    res = autotune._search(ctx, (("ss", autotune.SS_KNOBS),), measure, None)
    setting, ms = res["ss"]
    assert setting == [sqd.TUNE_SS_ROWS, 2, sqd.TUNE_SS_WAVES, 4]
    assert ms == pytest.approx(0.54)
    # the winner stays applied; reset restores every knob to automatic
    assert ctx.tune[sqd.TUNE_SS_ROWS] == 2 and ctx.tune[sqd.TUNE_SS_WAVES] == 4
    autotune.reset(ctx)
    assert all(ctx.tune[k] == 0 for k in autotune.ALL_KEYS)


def test_autotune_cache_round_trip(tmp_path, monkeypatch):
    from paper_2601_16169_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "cache.json"))
    assert autotune._load() == {}
    autotune._store("dev|sig", {"ss": [[0, 4, 3, 8], 0.1]})
    autotune._store("dev|sig2", {"ab": [[6, 1], 0.2]})
    got = autotune._load()
    assert got["dev|sig"]["ss"][0] == [0, 4, 3, 8] and "dev|sig2" in got
    (tmp_path / "cache.json").write_text("{not json")
    assert autotune._load() == {}
