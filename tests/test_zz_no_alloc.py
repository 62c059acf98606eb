"""The allocation-free ping + detection entry point against sonar_ping_detect
(needs an MI355X): identical volume bits and point clouds on two calls in a
row, the second with a smaller layout, and host-side rejection of sizes
beyond its scratch."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

from paper_2606_06130_amd import scenes as S

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU (it must not pass by skipping)")
    from paper_2606_06130_amd import sonar
    return torch, sonar


def _run_pair(torch, sonar, sc, cfg, pose):
    """Points and volume of sonar_ping_detect and of the allocation-free call."""
    ref = sonar.Detector(cfg)
    v_ref = sonar.alloc_outputs(cfg)["volume"]
    ref.ping_detect(sc, v_ref, pose)
    p_ref, n_ref = ref.fetch()
    det = sonar.Detector(cfg)
    v = sonar.alloc_outputs(cfg)["volume"]
    v.fill_(complex(float("nan"), 0.0))
    det.points.fill_(-1)
    det.count.fill_(-1)
    det.ping_detect_noalloc(sc, v, pose)
    p, n = det.fetch()
    torch.cuda.synchronize()
    assert torch.equal(v.view(torch.float32), v_ref.view(torch.float32))
    assert n == n_ref
    assert np.array_equal(p.view(np.int32), p_ref.view(np.int32))
    return n


def test_noalloc_matches_ping_detect_twice_smaller_second():
    torch, sonar = _gpu()
    mesh = S.scene_harbor()
    sc = sonar.Scene(mesh)
    cfg1, pose1 = S.sensor_harbor(), S.pose_harbor()
    n1 = _run_pair(torch, sonar, sc, cfg1, pose1)
    cfg2 = cfg1.replace(n_h=48, n_v=20, rays_per_beam=4, n_range=333)
    pose2 = S.pose((0.3, -1.0, -2.5), yaw=0.1, pitch_down=math.radians(30.0), ping=5)
    n2 = _run_pair(torch, sonar, sc, cfg2, pose2)
    print("no-alloc ping+detect: points", n1, n2, flush=True)
    sys.stdout.flush()
    assert n1 > 0 and n2 > 0


def test_noalloc_multipath_receive_binning_list_in_scratch():
    """Receive binning with several bounces: the moved-return list lives in
    the scratch too (atomics place those returns: compare to rounding)."""
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    sc = sonar.Scene(mesh)
    cfg = S.sensor_seabed_boxes().replace(max_bounces=3, k_d=0.7, k_s=0.3, n_range=512,
                                          flags=sonar.FLAG_RX_BEAMS)
    pose = S.pose_seabed_boxes()
    ref = sonar.Detector(cfg)
    v_ref = sonar.alloc_outputs(cfg)["volume"]
    ref.ping_detect(sc, v_ref, pose)
    det = sonar.Detector(cfg)
    v = sonar.alloc_outputs(cfg)["volume"]
    det.ping_detect_noalloc(sc, v, pose)
    torch.cuda.synchronize()
    a = v.cpu().numpy().ravel()
    b = v_ref.cpu().numpy().ravel()
    assert np.abs(a - b).max() <= 1e-6 * np.abs(b).max()


def test_noalloc_rejects_sizes_beyond_scratch():
    torch, sonar = _gpu()
    sc = sonar.Scene(S.scene_seabed_boxes())
    cfg = S.sensor_harbor().replace(n_h=512, n_v=256)          # 131,072 beams: 17 MB of detection workspace
    det_cfg = cfg.replace(n_h=8, n_v=8)
    det = sonar.Detector(det_cfg)
    p = sonar.params_of(cfg)
    q = sonar.pose_of(S.pose_harbor())
    st = sonar.lib().sonar_ping_detect_noalloc(sc.handle, C.byref(p), C.byref(q), C.byref(det.cfar), None, None, 0,
                                               None, None)
    assert st == sonar.SONAR_E_INVALID
    assert b"scratch" in sonar.lib().sonar_last_error()
