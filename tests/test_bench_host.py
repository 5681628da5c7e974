"""Host-side pieces of bench.py: the tile-shape argument, the lookup of stored
counter traffic, and the one-GPU guard (no device needed)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_shape_argument_round_trip():
    assert bench.parse_shape("16/16") == dict(band_y=16, band_y_small=16, instance_bands={}, solo_max_nodes=0,
                                              rounds_per_graph=0, stagger=0)
    L = bench.parse_shape("32/8:5=4,502=8;solo=9216;rpg=32;stagger=1")
    assert L == dict(band_y=32, band_y_small=8, instance_bands={5: 4, 502: 8}, solo_max_nodes=9216,
                     rounds_per_graph=32, stagger=1)
    assert bench.shape_text(L) == "32/8:5=4,502=8;solo=9216;rpg=32;stagger=1"
    assert bench.shape_text(bench.parse_shape("16/16:7=4")) == "16/16:7=4"
    assert bench.shape_text(bench.parse_shape("16/4;rpg=8")) == "16/4;rpg=8"


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
    # another workload line of the same kernel: only the measured ratio carries over
    assert bench.profile_traffic("k_round<StoreF16S>") is None   # no algorithmic bytes recorded
    line["algorithmic_bytes"] = 5
    (prof / "p.md").write_text("bench-traffic: " + json.dumps(line) + "\n")
    assert bench.profile_traffic("k_round<StoreF16S>") == {"workload": "w", "traffic_over_algorithmic": 1.4}
    line["src_sha"] = "0" * 16   # counters taken on other kernel sources
    (prof / "p.md").write_text("bench-traffic: " + json.dumps(line) + "\n")
    assert bench.stored_traffic("k_round<StoreF16S>", "w") is None
    assert bench.profile_traffic("k_round<StoreF16S>") is None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_trace_and_counter_summaries_take_the_last_dispatches(tmp_path):
    """The reducers of rocprofv3 CSV output that turn a profile into the
    figures of profiles/: durations and counters of the last N dispatches of
    one kernel, in dispatch order."""
    kt = tmp_path / "kernel_trace.csv"
    rows = ["Kind,Dispatch_Id,Kernel_Name,Start_Timestamp,End_Timestamp"]
    t = 0
    for d in range(10):
        name = "k_round<lbm::StoreF16S>(lbm::Ctx)" if d % 2 == 0 else "k_finalize(lbm::Ctx)"
        rows.append(f"KERNEL_DISPATCH,{d},\"{name}\",{t},{t + 1000 * (d + 1)}")
        t += 100000
    kt.write_text("\n".join(rows) + "\n")
    s = bench.trace_summary(str(kt), "k_round<lbm::StoreF16S>", 3)
    assert s["dispatches_in_trace"] == 5 and s["taken"] == 3
    assert s["mean_us"] == (5 + 7 + 9) / 3
    cc = tmp_path / "counter_collection.csv"
    rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    for d in range(6):
        rows.append(f"{d},\"k_round<lbm::StoreF16S>(lbm::Ctx)\",FETCH_SIZE,{100 * d}")
        rows.append(f"{d},\"k_round<lbm::StoreF16S>(lbm::Ctx)\",WRITE_SIZE,{7 * d}")
    cc.write_text("\n".join(rows) + "\n")
    c = bench.counter_summary(str(cc), "k_round<lbm::StoreF16S>", 2, "FETCH_SIZE")
    assert c["taken"] == 2 and c["mean"] == 450.0
