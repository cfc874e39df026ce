"""Host-side checks of the benchmark's bookkeeping (no GPU): the committed
HBM-traffic summaries parse (and give their total while they name the current
kernel sources), a changed source gives no traffic figure, the flops-per-pair counts are the stated ones,
and a request for more than one GPU stops before any device work."""
import os
import re
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("key", sorted(bench.PROFILE_TRAFFIC))
def test_traffic_profiles_parse_and_match_sources(key):
    path = os.path.join(ROOT, "profiles", bench.PROFILE_TRAFFIC[key])
    assert os.path.exists(path), path
    text = open(path).read()
    fetch = float(re.search(r"fetch_bytes_per_launch:\s*(\S+)", text).group(1))
    write = float(re.search(r"write_bytes_per_launch:\s*(\S+)", text).group(1))
    assert fetch > 0 and write >= 0
    total = bench.traffic_from_profile(key)
    if total is None:
        pytest.skip(f"{path} was taken on other kernel sources: the benchmark reports no traffic for it")
    assert total == pytest.approx(fetch + write, rel=1e-3)
    assert total > 0


def test_changed_source_gives_no_traffic(monkeypatch):
    key = "fp64"
    assert bench.traffic_from_profile(key) is not None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k: "0" * 16)
    assert bench.traffic_from_profile(key) is None


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    src = tmp_path / "paper_1909_11085_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "a.hip").write_text("int f() { return 1; }  // one\n/* block */\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.PROFILE_SOURCES, "t", ("a.hip",))
    h0 = bench.kernel_source_hash("t")
    (src / "a.hip").write_text("int f() {\n  return 1;  // another comment\n}\n")
    assert bench.kernel_source_hash("t") == h0
    (src / "a.hip").write_text("int f() { return 2; }\n")
    assert bench.kernel_source_hash("t") != h0


def test_flop_counts():
    # single layer 29 per ordered pair, 23 per interaction each pair once
    # (46 per unordered pair), double layer 30
    assert (bench.FLOPS_PER_PAIR_SL, bench.FLOPS_PER_PAIR_SL_SYM, bench.FLOPS_PER_PAIR_DL) == (29, 23, 30)
    assert bench.flops_sl("fp64", False) == 23 and bench.flops_sl("fp64", True) == 29
    assert bench.flops_sl("mixed", False) == 29


def test_more_than_one_gpu_stops():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "exactly one GPU" in (r.stdout + r.stderr)
