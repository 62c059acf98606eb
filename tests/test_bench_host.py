"""Host logic of the benchmark's CPU-baseline leg: the sample walks ping
after ping along the job's poses and counts only the beams it traced."""
import re
import time

import numpy as np

import bench
import oracle
from paper_2606_06130_amd import scenes as S


def test_cpu_baseline_counts_traced_beams(monkeypatch):
    mesh = S.scene_seabed_boxes()
    cfg = S.sensor_seabed_boxes()
    poses = [S.pose_seabed_boxes(), S.pose_seabed_boxes_level(), S.pose_seabed_boxes()]
    calls = []

    def fake_trace(scene, c, pose, beams, threads=1, want_all=False):
        calls.append((threads, pose, np.asarray(beams).copy()))
        time.sleep(0.002)
        return {}

    monkeypatch.setattr(oracle, "trace_beams", fake_trace)
    res = bench.cpu_baseline(mesh, cfg, poses, budget_s=0.3, single_budget_s=0.05, brute_budget_s=0.05)
    threads = res["cores"]
    # the main leg: the first run of calls at `threads` threads, up to its budget
    first_leg = []
    for t, p, b in calls:
        if t != threads:
            break
        first_leg.append((p, b))
    traced = sum(len(b) for _, b in first_leg)
    m = re.match(r"(\d+) beams", res["sample"])
    assert m and int(m.group(1)) == traced
    assert traced > cfg.n_beams          # the budget outlasts one ping: it moved on to the next pose
    done = 0
    for p, b in first_leg:
        ping, first = divmod(done, cfg.n_beams)
        assert p is poses[ping % len(poses)]
        assert len(b) >= 1 and first + len(b) <= cfg.n_beams      # never past the end of a ping
        done += len(b)
