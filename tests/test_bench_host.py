"""Host logic of bench.py (no GPU): the HBM-traffic lookup in the committed
counter summary and the --gpus guard."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _summary(blocks):
    parts = ["# summary\n\nprose\n"]
    for b in blocks:
        parts.append("```\n" + "\n".join(f"{k}: {v}" for k, v in b.items()) + "\n```\n\nmore prose\n")
    return "".join(parts)


def _block(shape, sha, fetch, write, fs=2.0, ws=1.0, kernel="k_gsrb<double>"):
    return {"kernel": kernel, "shape": " ".join(str(x) for x in shape), "source_sha256": sha,
            "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write,
            "fetch_scale": fs, "write_scale": ws}


def test_traffic_lookup_picks_the_matching_block(tmp_path, monkeypatch):
    sha = bench.kernel_source_sha256()
    f = tmp_path / "traffic.md"
    f.write_text(_summary([_block((32, 8, 2, 2, 0), sha, 100.0, 50.0),
                           _block((32, 4, 2, 2, 0), sha, 200.0, 60.0),
                           _block((32, 2, 2, 2, 0), "0" * 64, 300.0, 70.0)]))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(f))
    assert bench.measured_traffic("k_gsrb<double>", (32, 8, 2, 2, 0)) == (100 * 2 + 50) * 1024
    assert bench.measured_traffic("k_gsrb<double>", (32, 4, 2, 2, 0)) == (200 * 2 + 60) * 1024
    # taken on other kernel sources, another shape, another kernel: no figure
    assert bench.measured_traffic("k_gsrb<double>", (32, 2, 2, 2, 0)) is None
    assert bench.measured_traffic("k_gsrb<double>", (64, 8, 2, 2, 0)) is None
    assert bench.measured_traffic("k_sweep<double>", (32, 8, 2, 2, 0)) is None


def test_traffic_lookup_keys_on_the_class_table(tmp_path, monkeypatch):
    """A block with a `classes:` line matches only a run with that per-class table; a
    block without one matches only the uniform table."""
    sha = bench.kernel_source_sha256()
    cls = dict(_block((32, 8, 2, 2, 0), sha, 400.0, 80.0), classes="64 64 4 2")
    f = tmp_path / "traffic.md"
    f.write_text(_summary([_block((32, 8, 2, 2, 0), sha, 100.0, 50.0), cls]))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(f))
    assert bench.measured_traffic("k_gsrb<double>", (32, 8, 2, 2, 0)) == (100 * 2 + 50) * 1024
    assert bench.measured_traffic("k_gsrb<double>", (32, 8, 2, 2, 0), {}) == (100 * 2 + 50) * 1024
    assert (bench.measured_traffic("k_gsrb<double>", (32, 8, 2, 2, 0), {"64": [64, 4, 2]})
            == (400 * 2 + 80) * 1024)
    assert bench.measured_traffic("k_gsrb<double>", (32, 8, 2, 2, 0), {"64": [32, 8, 4]}) is None
    assert bench.measured_traffic("k_gsrb<double>", (32, 8, 2, 2, 0),
                                  {"64": [64, 4, 2], "32": [32, 8, 2]}) is None


def test_traffic_lookup_tolerates_missing_or_broken_summaries(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "absent.md"))
    assert bench.measured_traffic("k_gsrb<double>", (32, 8, 2, 2, 0)) is None
    f = tmp_path / "broken.md"
    f.write_text("```\nkernel: k_gsrb<double>\nshape: 32 8 two 2 0\n```\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(f))
    assert bench.measured_traffic("k_gsrb<double>", (32, 8, 2, 2, 0)) is None


def test_committed_summary_parses():
    """The committed summary holds at least one well-formed block."""
    text = open(bench.TRAFFIC_PROFILE).read()
    blocks = text.split("```")[1::2]
    assert any("hbm_bytes_per_launch" in b and "source_sha256" in b for b in blocks)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
