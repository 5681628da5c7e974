"""Host-side pieces of bench.py: the tile-shape argument, the lookup of stored
counter traffic, and the one-GPU guard (no device needed)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_shape_argument_round_trip():
    assert bench.parse_shape("16/16") == (16, 16, {})
    assert bench.parse_shape("32/8:5=4,502=8") == (32, 8, {5: 4, 502: 8})


def test_stored_traffic_needs_kernel_digest_and_workload_to_match(tmp_path, monkeypatch):
    sha = bench.src_digest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    line = {"kernel": "k_round<StoreF16S>", "src_sha": sha, "workload": "w", "bytes_per_launch": 7}
    (prof / "p.md").write_text("text\nbench-traffic: " + json.dumps(line) + "\n")
    # profiles from the temporary tree, kernel sources from this one
    monkeypatch.setattr(bench, "src_digest", lambda: sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_traffic("k_round<StoreF16S>", "w")["bytes_per_launch"] == 7
    assert bench.stored_traffic("k_round<StoreF16S>", "other workload") is None
    assert bench.stored_traffic("k_round<StoreF32>", "w") is None
    line["src_sha"] = "0" * 16   # counters taken on other kernel sources
    (prof / "p.md").write_text("bench-traffic: " + json.dumps(line) + "\n")
    assert bench.stored_traffic("k_round<StoreF16S>", "w") is None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
