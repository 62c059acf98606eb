"""Pings through a piecewise-linear sound-speed profile on the GPU against the
FP64 oracle, through the C-ABI: single bounce, and several bounces with each
later vertex returning along its first-arriving eigenray (needs an MI355X)."""
import math

import numpy as np
import pytest

from paper_2606_06130_amd import scenes as S
from tests import meshes as M
from tests.test_gpu_parity import _gpu, _log, assert_parity, run_parity

pytestmark = pytest.mark.gpu

# speed falling with depth at four different rates (0.05-0.48 /s, inside the
# one-chord-per-layer bound): rays refract across four knots
KNOTS = ((-9.0, 1497.0), (-6.0, 1498.2), (-3.0, 1499.0), (-0.5, 1500.2), (1.5, 1500.3))
# for the surface-and-wall scene: four gradients between 0.05 and 0.48 /s
# (return rays turn above the span), and a speed minimum at -3 m (they turn
# above or below it)
KNOTS_MP = ((-8.0, 1497.1), (-5.0, 1498.5), (-2.0, 1498.8), (0.5, 1500.0), (2.5, 1500.1))
KNOTS_CHANNEL = ((-8.0, 1500.0), (-3.0, 1498.0), (2.5, 1499.5))


def _surface_wall():
    surf = M.mesh_from([M.big_triangle_z(2.0)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    rng = np.random.Generator(np.random.PCG64(1))
    wall = M.plane_grid_x(8.0, -6.0, 6.0, -8.0, 2.0, 40, rng)
    mesh = M.concat(surf, wall)
    mesh.name = "surface_wall_layered"
    return mesh


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


@pytest.mark.parametrize("knots,K", [(KNOTS_MP, 2), (KNOTS_MP, 3), (KNOTS_CHANNEL, 3)])
def test_surface_wall_layered_multipath(knots, K):
    """Pressure-release surface and a wall, several bounces through the
    layers: outgoing legs piece by piece, eigenray connections (direct and
    turning) with their occlusion walked one circle per layer."""
    cfg = S.SensorConfig(n_h=32, n_v=16, rays_per_beam=4, n_range=1024, max_bounces=K, k_d=0.7, k_s=0.3,
                         vfov=math.radians(60), ssp=knots)
    res, g, orc = run_parity(_surface_wall(), cfg, S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10)))
    assert_parity(res, K)
    assert res["im_energy"] > 0 and (orc["bin"][:, 1] >= 0).sum() > 500


def test_layered_multipath_receive_binning_and_pattern():
    """Returns of later bounces binned by their arrival direction (the
    eigenray's arrival at the sensor), through the workspace call."""
    cfg = S.SensorConfig(n_h=32, n_v=16, rays_per_beam=4, n_range=1024, max_bounces=3, k_d=0.7, k_s=0.3,
                         vfov=math.radians(60), ssp=KNOTS_CHANNEL, flags=1 | 2)
    res, g, orc = run_parity(_surface_wall(), cfg, S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10)))
    assert_parity(res, 3)
    moved = (orc["bin"][:, 1:] >= 0) & (orc["rxb"][:, 1:] != (np.arange(len(orc["rxb"])) // 4)[:, None])
    assert moved.sum() > 50


def test_layered_multipath_drawn_continuations():
    cfg = S.SensorConfig(n_h=32, n_v=16, rays_per_beam=4, n_range=1024, max_bounces=3, k_d=0.7, k_s=0.3,
                         vfov=math.radians(60), ssp=KNOTS_CHANNEL, seed=21, flags=4)
    res, g, orc = run_parity(_surface_wall(), cfg, S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10)))
    assert_parity(res, 3)
    assert res["im_energy"] > 0


def test_layered_multipath_knots_on_one_line_equal_the_linear_profile():
    torch, sonar = _gpu()
    sc = sonar.Scene(_surface_wall())
    pose = S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10))
    base = S.SensorConfig(n_h=32, n_v=16, rays_per_beam=4, n_range=1024, max_bounces=3, k_d=0.7, k_s=0.3,
                          vfov=math.radians(60))
    lin = base.replace(c_grad=0.05)
    lay = base.replace(ssp=tuple((z, 1500.0 + 0.05 * z) for z in (-9.0, -6.5, -3.25, -1.0, 0.5, 4.0)))
    a = sonar.ping(sc, lin, pose, record=True, incoh=True)
    b = sonar.ping(sc, lay, pose, record=True, incoh=True)
    torch.cuda.synchronize()
    assert sc.status() == 0
    assert (a["tri"] == b["tri"]).float().mean().item() > 0.999
    assert (a["bin"] == b["bin"]).float().mean().item() > 0.999
    for key in ("volume", "incoh"):
        va, vb = a[key].cpu().numpy(), b[key].cpu().numpy()
        assert np.linalg.norm(va - vb) <= 2e-3 * np.linalg.norm(va), key


def test_harbor_layered_multipath_full_size_sampled_beams():
    """The harbor multipath scene (1,991,680 triangles, 3 bounces, 256 x 128
    beams x 16 rays) through the layered profile, as one launch; 40 beams
    compared ray by ray, bounce by bounce."""
    mesh = S.scene_harbor_multipath()
    cfg, pose = S.sensor_harbor_multipath().replace(c_grad=0.0, ssp=KNOTS), S.pose_harbor()
    rng = np.random.Generator(np.random.PCG64(44))
    beams = np.sort(rng.choice(cfg.n_beams, 40, replace=False))
    res, g, orc = run_parity(mesh, cfg, pose, beams=beams)
    assert_parity(res, 3)
    assert res["im_energy"] > 0


def test_layered_profile_rejections():
    torch, sonar = _gpu()
    sc = sonar.Scene(S.scene_seabed_boxes())
    pose = S.pose_seabed_boxes()
    cfg = S.sensor_seabed_boxes().replace(ssp=KNOTS)
    # receive binning with several bounces needs the workspace call
    import ctypes as C
    bad = cfg.replace(max_bounces=2, flags=2)
    out = sonar.alloc_outputs(bad)
    st = sonar.lib().sonar_ping_ssp(sc.handle, C.byref(sonar.params_of(bad)), C.byref(sonar.pose_of(pose)),
                                    C.byref(sonar.ssp_of(bad.ssp)), out["volume"].data_ptr(), None, None, None, None,
                                    None)
    assert st == sonar.SONAR_E_INVALID
    for bad, status in ((cfg.replace(ssp=((0.0, 1500.0), (-1.0, 1490.0))), sonar.SONAR_E_INVALID),
                        (cfg.replace(ssp=((0.0, 1500.0),)), sonar.SONAR_E_INVALID),
                        (cfg.replace(ssp=((-1.0, 1500.0), (0.0, 0.0))), sonar.SONAR_E_INVALID),
                        (cfg.replace(ssp=((-1.0, 1400.0), (0.0, 1500.0))), sonar.SONAR_E_UNSUPPORTED)):
        with pytest.raises(sonar.SonarError) as e:
            sonar.ping(sc, bad, pose)
        assert e.value.status == status, (bad.ssp, bad.max_bounces)
    with pytest.raises(sonar.SonarError):
        sonar.Detector(cfg).ping_detect(sc, sonar.alloc_outputs(cfg)["volume"], pose)
    with pytest.raises(sonar.SonarError):
        sonar.Batch(sc, [(cfg, pose), (cfg.replace(ssp=KNOTS_MP), pose)])     # one profile per batch


@pytest.mark.parametrize("K", [1, 3])
def test_layered_batch_equals_single_pings(K):
    """A batch through one layered profile (mixed layouts and poses, one
    persistent launch) writes the same volumes, bit for bit, as single pings."""
    torch, sonar = _gpu()
    sc = sonar.Scene(_surface_wall())
    base = S.SensorConfig(n_range=1024, max_bounces=K, k_d=0.7, k_s=0.3, vfov=math.radians(60), ssp=KNOTS_CHANNEL)
    items = [(base.replace(n_h=nh, n_v=nv, rays_per_beam=nr),
              S.pose((0.3 * i, -0.2 * i, -0.5 * i), pitch_down=math.radians(-10 + 3 * i), ping=i))
             for i, (nh, nv, nr) in enumerate([(32, 16, 4), (16, 8, 16), (33, 7, 1), (64, 32, 4)])]
    b = sonar.Batch(sc, items)
    assert b.plan.arc == 2
    b.run()
    torch.cuda.synchronize()
    assert sc.status() == 0
    for i, (cfg, pose) in enumerate(items):
        ref = sonar.ping(sc, cfg, pose)["volume"]
        torch.cuda.synchronize()
        assert torch.equal(b.volumes[i].view(torch.float32), ref.view(torch.float32)), i
        assert torch.count_nonzero(ref).item() > 0
