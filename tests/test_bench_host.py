"""Host logic of the benchmark script, no GPU: the one-GPU refusal, the
latency percentile, the JSON line's keys, and the rule that a stored HBM
traffic figure is used only while the kernel source it was taken on is
unchanged."""
import hashlib
import json
import math
import os
import subprocess
import sys
import types

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for n in (2, 8):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                           capture_output=True, text=True, timeout=60)
        assert r.returncode == 2
        assert "one GPU" in r.stderr and r.stdout == ""


def test_percentile_is_nearest_rank():
    xs = list(range(1, 101))[::-1]
    assert bench.percentile(xs, 50) == 50
    assert bench.percentile(xs, 99) == 99
    assert bench.percentile(xs, 100) == 100
    assert bench.percentile([7.0], 99) == 7.0
    assert bench.percentile([3, 1, 2], 50) == 2
    assert math.isnan(bench.percentile([], 50))


def test_json_line_carries_the_contract_keys(capsys):
    args = types.SimpleNamespace(steps=7, warmup=2)
    bench.form_line(args, "updates_per_s", 123.5, 4.25, {"config": {"workload": "w"}})
    line = capsys.readouterr().out.strip().splitlines()
    assert len(line) == 1
    out = json.loads(line[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config"):
        assert k in out
    assert out["n_gpus"] == 1 and out["steps"] == 7 and out["warmup"] == 2
    assert out["value"] == 123.5 and out["ms_per_step"] == 4.25
    assert out["higher_is_better"] is True and out["vs_baseline"] is None
    assert out["config"] == {"workload": "w"}


def test_stored_traffic_only_for_the_source_it_was_taken_on(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2308_14493_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = csrc / "k.hip"
    src.write_bytes(b"kernel text one\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    summary = tmp_path / "profiles" / "pmc_k.md"
    summary.write_text("kernel: k\nsource_sha256_prefix: %s\ntraffic_bytes_per_launch: 1.5e9\n" % sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k.hip", "pmc_k.md") == 1.5e9
    src.write_bytes(b"kernel text two\n")
    assert bench.measured_traffic("k.hip", "pmc_k.md") is None
    src.write_bytes(b"kernel text one\n")
    summary.write_text("kernel: k\nsource_sha256_prefix: %s\n" % sha)
    assert bench.measured_traffic("k.hip", "pmc_k.md") is None
    assert bench.measured_traffic("k.hip", "missing.md") is None
