"""Single-bounce pings through a piecewise-linear sound-speed profile on the
GPU against the FP64 oracle, through the C-ABI (needs an MI355X)."""
import math

import numpy as np
import pytest

from paper_2606_06130_amd import scenes as S
from tests.test_gpu_parity import _gpu, _log, assert_parity, run_parity

pytestmark = pytest.mark.gpu

# speed falling with depth at four different rates (0.05-0.48 /s, inside the
# one-chord-per-layer bound): rays refract across four knots
KNOTS = ((-9.0, 1497.0), (-6.0, 1498.2), (-3.0, 1499.0), (-0.5, 1500.2), (1.5, 1500.3))


@pytest.mark.parametrize("n_h,n_v,n_r", [(16, 8, 4), (33, 17, 16), (64, 32, 1)])
def test_seabed_boxes_layered_profile(n_h, n_v, n_r):
    mesh = S.scene_seabed_boxes()
    cfg = S.sensor_seabed_boxes().replace(n_h=n_h, n_v=n_v, rays_per_beam=n_r, n_range=512, ssp=KNOTS)
    res, g, orc = run_parity(mesh, cfg, S.pose_seabed_boxes())
    assert_parity(res)
    assert res["energy"] > 0


def test_knots_on_one_line_equal_the_linear_profile_on_the_gpu():
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    pose = S.pose_seabed_boxes()
    sc = sonar.Scene(mesh)
    base = S.sensor_seabed_boxes().replace(n_h=32, n_v=16, rays_per_beam=4, n_range=512)
    lin = base.replace(c_grad=0.05)
    lay = base.replace(ssp=tuple((z, 1500.0 + 0.05 * z) for z in (-9.0, -6.5, -3.25, -1.0, 0.5, 4.0)))
    a = sonar.ping(sc, lin, pose, record=True)
    b = sonar.ping(sc, lay, pose, record=True)
    torch.cuda.synchronize()
    assert sc.status() == 0
    same = (a["tri"] == b["tri"]).float().mean().item()
    assert same > 0.999                                  # chord splits can move edge rays only
    va, vb = a["volume"].cpu().numpy(), b["volume"].cpu().numpy()
    assert np.linalg.norm(va - vb) <= 1e-3 * np.linalg.norm(va)


def test_harbor_layered_full_size_sampled_beams():
    """The harbor ping (601,088 triangles, 256 x 128 beams x 16 rays) through
    the layered profile, as one launch; 64 beams compared ray by ray."""
    mesh = S.scene_harbor()
    cfg, pose = S.sensor_harbor().replace(ssp=KNOTS), S.pose_harbor()
    rng = np.random.Generator(np.random.PCG64(43))
    beams = np.sort(rng.choice(cfg.n_beams, 64, replace=False))
    res, g, orc = run_parity(mesh, cfg, pose, beams=beams)
    assert_parity(res)


def test_layered_profile_rejections():
    torch, sonar = _gpu()
    sc = sonar.Scene(S.scene_seabed_boxes())
    pose = S.pose_seabed_boxes()
    cfg = S.sensor_seabed_boxes().replace(ssp=KNOTS)
    for bad, status in ((cfg.replace(max_bounces=2), sonar.SONAR_E_UNSUPPORTED),
                        (cfg.replace(ssp=((0.0, 1500.0), (-1.0, 1490.0))), sonar.SONAR_E_INVALID),
                        (cfg.replace(ssp=((0.0, 1500.0),)), sonar.SONAR_E_INVALID),
                        (cfg.replace(ssp=((-1.0, 1500.0), (0.0, 0.0))), sonar.SONAR_E_INVALID),
                        (cfg.replace(ssp=((-1.0, 1400.0), (0.0, 1500.0))), sonar.SONAR_E_UNSUPPORTED)):
        with pytest.raises(sonar.SonarError) as e:
            sonar.ping(sc, bad, pose)
        assert e.value.status == status, (bad.ssp, bad.max_bounces)
    with pytest.raises(sonar.SonarError):
        sonar.Detector(cfg).ping_detect(sc, sonar.alloc_outputs(cfg)["volume"], pose)
    with pytest.raises(sonar.SonarError):
        sonar.Batch(sc, [(cfg, pose)])
