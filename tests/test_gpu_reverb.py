"""Water-column reverberation and receiver noise on the GPU against the FP64
oracle, through the C-ABI (needs an MI355X)."""
import math
import sys

import numpy as np
import pytest

from oracle import reverb as R
from paper_2606_06130_amd import scenes as S

pytestmark = pytest.mark.gpu

TOL = 1e-5          # relative L2: FP32 power law and Box-Muller against FP64


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU (it must not pass by skipping)")
    from paper_2606_06130_amd import sonar
    return torch, sonar


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.complex128) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n_h,n_v,n_range,sv,noise,ping,seed", [
    (32, 16, 256, -40.0, 0.0, 0, 1), (32, 16, 256, -60.0, 1e-12, 7, 99), (7, 3, 1000, -20.0, 1e-9, 1, 5),
    (64, 1, 33, -45.0, 0.0, 123456, 2 ** 63 + 3), (1, 1, 1, -30.0, 1e-10, 0, 0)])
def test_small_volumes_match_oracle(n_h, n_v, n_range, sv, noise, ping, seed):
    torch, sonar = _gpu()
    cfg = S.SensorConfig(n_h=n_h, n_v=n_v, n_range=n_range, r_min=0.4, r_max=20.0, abs_db_per_m=0.3)
    pose = S.pose((0.0, 0.0, -2.0), ping=ping)
    rng = np.random.Generator(np.random.PCG64(n_range))
    x = ((rng.normal(size=(n_v * n_h, n_range)) + 1j * rng.normal(size=(n_v * n_h, n_range))) * 1e-4).astype(
        np.complex64)
    print("reverb", n_h, n_v, n_range, sv, noise, ping, flush=True)
    xd = torch.from_numpy(x).cuda().view(n_v, n_h, n_range)
    sonar.add_reverb(xd, cfg, pose, sv, noise, seed)
    torch.cuda.synchronize()
    got = xd.view(-1, n_range).cpu().numpy()
    want = R.add(x.astype(np.complex128), cfg, ping, sv, noise, seed)
    assert _rel(got - x, want - x) <= TOL


def test_harbor_size_sampled_beams():
    """The harbor layout (32,768 beams x 1,024 bins) in the benchmark's launch
    configuration: sampled beams against the oracle, empty input."""
    torch, sonar = _gpu()
    cfg, pose = S.sensor_harbor(), S.pose_harbor()
    bv, bh = sonar.beams_of(cfg)
    v = torch.zeros((bv, bh, cfg.n_range), dtype=torch.complex64, device="cuda")
    sonar.add_reverb(v, cfg, pose, -50.0, 1e-13, 2024)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(8))
    nb = bv * bh
    beams = np.concatenate([[0, nb - 1], rng.choice(nb, 62, replace=False)])
    got = v.view(nb, -1)[torch.from_numpy(beams).cuda()].cpu().numpy()
    want = R.add(np.zeros((len(beams), cfg.n_range)), cfg, pose.ping, -50.0, 1e-13, 2024, beams=beams)
    assert _rel(got, want) <= TOL
    # mean power per bin over all beams follows the mean-power law
    p = (v.view(nb, -1).abs() ** 2).mean(dim=0).double().cpu().numpy()
    P = R.mean_power(cfg, np.arange(nb), np.arange(cfg.n_range), -50.0, 1e-13).mean(axis=0)
    assert np.all(np.abs(p / P - 1.0) < 6 / math.sqrt(nb))


def test_ping_reverb_then_detect_runs():
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    cfg, pose = S.sensor_seabed_boxes(), S.pose_seabed_boxes()
    sc = sonar.Scene(mesh)
    vol = sonar.ping(sc, cfg, pose)["volume"]
    sonar.add_reverb(vol, cfg, pose, -60.0, 1e-14, 3)
    det = sonar.Detector(cfg)
    det(vol, pose)
    pts, n = det.fetch()
    torch.cuda.synchronize()
    assert sc.status() == 0 and n > 0
