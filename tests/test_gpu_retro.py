"""Retro-chain returns (a later vertex scattering back along its outgoing
chain reversed) on the GPU against the FP64 oracle, through the C-ABI (needs
an MI355X)."""
import math

import numpy as np
import pytest

from paper_2606_06130_amd import scenes as S
from tests import meshes as M
from tests.test_gpu_parity import _gpu, assert_parity, run_parity

pytestmark = pytest.mark.gpu

RETRO = 8
KNOTS = ((-8.0, 1497.1), (-5.0, 1498.5), (-2.0, 1498.8), (0.5, 1500.0), (2.5, 1500.1))


def _surface_wall():
    surf = M.mesh_from([M.big_triangle_z(2.0)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    wall = M.plane_grid_x(8.0, -6.0, 6.0, -8.0, 2.0, 40, np.random.Generator(np.random.PCG64(1)))
    mesh = M.concat(surf, wall)
    mesh.name = "surface_wall_retro"
    return mesh


def _cfg(**kw):
    base = dict(n_h=32, n_v=16, rays_per_beam=4, n_range=1024, max_bounces=3, k_d=0.7, k_s=0.3,
                vfov=math.radians(60), flags=RETRO)
    base.update(kw)
    return S.SensorConfig(**base)


POSE = S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10))


@pytest.mark.parametrize("K,g", [(2, 0.0), (3, 0.0), (3, 0.05), (4, 0.05)])
def test_surface_wall_retro_chain(K, g):
    res, out, orc = run_parity(_surface_wall(), _cfg(max_bounces=K, c_grad=g), POSE)
    assert_parity(res, K)
    assert res["retro_returns"] > 300


def test_retro_chain_layered_profile():
    res, out, orc = run_parity(_surface_wall(), _cfg(ssp=KNOTS), POSE)
    assert_parity(res, 3)
    assert res["retro_returns"] > 300


@pytest.mark.parametrize("flags", [RETRO | 1, RETRO | 4])
def test_retro_chain_with_pattern_and_drawn_continuations(flags):
    res, out, orc = run_parity(_surface_wall(), _cfg(flags=flags, seed=13), POSE)
    assert_parity(res, 3)


def test_retro_chain_with_receive_binning():
    res, out, orc = run_parity(_surface_wall(), _cfg(flags=RETRO | 2 | 1), POSE)
    assert_parity(res, 3)
    assert res["retro_returns"] > 300


def test_retro_chain_adds_only_its_returns():
    torch, sonar = _gpu()
    sc = sonar.Scene(_surface_wall())
    on = sonar.ping(sc, _cfg(), POSE, record=True, incoh=True)
    off = sonar.ping(sc, _cfg(flags=0), POSE, record=True, incoh=True)
    torch.cuda.synchronize()
    for key in ("tri", "bin", "vis", "amp"):
        assert torch.equal(on[key], off[key]), key
    assert torch.equal(on["incoh"][0], off["incoh"][0])
    # the volume gains the retro returns (binned per beam in FP64 here)
    rbin = on["rbin"].cpu().numpy()
    ramp = on["ramp"].cpu().numpy()
    cfg = _cfg()
    extra = np.zeros((cfg.n_beams, cfg.n_range), complex)
    for ray, k in zip(*np.nonzero(rbin >= 0)):
        extra[ray // cfg.rays_per_beam, rbin[ray, k]] += ramp[ray, k]
    d = (on["volume"] - off["volume"]).cpu().numpy().reshape(cfg.n_beams, -1)
    assert np.linalg.norm(d - extra) <= 1e-5 * np.linalg.norm(extra)


def test_fused_detection_with_retro_chain_matches_separate():
    """sonar_ping_detect with retro-chain slots in the fused CFAR equals
    sonar_ping + sonar_detect (the same volume bits, the same points up to
    decisions at their threshold)."""
    torch, sonar = _gpu()
    sc = sonar.Scene(_surface_wall())
    cfg = _cfg()
    v1 = sonar.ping(sc, cfg, POSE)["volume"]
    d1 = sonar.Detector(cfg)
    d1(v1, POSE)
    p1, n1 = d1.fetch()
    v2 = torch.empty_like(v1)
    d2 = sonar.Detector(cfg)
    d2.ping_detect(sc, v2, POSE)
    p2, n2 = d2.fetch()
    assert torch.equal(v1.view(torch.float32), v2.view(torch.float32))
    assert n1 > 0 and abs(n1 - n2) <= 2
    k1 = set(zip(p1["beam"].tolist(), p1["bin"].tolist()))
    k2 = set(zip(p2["beam"].tolist(), p2["bin"].tolist()))
    assert len(k1 ^ k2) <= 4


def test_retro_chain_rejections():
    torch, sonar = _gpu()
    sc = sonar.Scene(_surface_wall())
    with pytest.raises(sonar.SonarError) as e:
        sonar.Batch(sc, [(_cfg(), POSE), (_cfg(flags=0), POSE)])          # all pings or none
    assert e.value.status == sonar.SONAR_E_INVALID
    with pytest.raises(sonar.SonarError) as e:
        sonar.ping(sc, _cfg(), POSE, record=True, stats=True)
    assert e.value.status == sonar.SONAR_E_UNSUPPORTED
    for K, most in ((3, 3328), (4, 3584)):
        with pytest.raises(sonar.SonarError) as e:
            sonar.ping(sc, _cfg(max_bounces=K, n_range=most + 2), POSE)
        assert e.value.status == sonar.SONAR_E_UNSUPPORTED
        sonar.ping(sc, _cfg(max_bounces=K, n_range=most), POSE)
    sonar.ping(sc, _cfg(max_bounces=2, n_range=4096), POSE)
    sonar.ping(sc, _cfg(max_bounces=1), POSE)                 # one bounce: nothing to retrace
    torch.cuda.synchronize()
    assert sc.status() == 0


def test_harbor_multipath_retro_chain_full_size_sampled_beams():
    """The harbor multipath ping (1,991,680 triangles, 3 bounces, 256 x 128
    beams x 16 rays) with retro-chain returns, as one launch of the
    benchmark's configuration; 40 beams compared ray by ray."""
    mesh = S.scene_harbor_multipath()
    cfg, pose = S.sensor_harbor_multipath().replace(flags=RETRO), S.pose_harbor()
    rng = np.random.Generator(np.random.PCG64(45))
    beams = np.sort(rng.choice(cfg.n_beams, 40, replace=False))
    res, out, orc = run_parity(mesh, cfg, pose, beams=beams)
    assert_parity(res, 3)
    assert res["retro_returns"] > 50


@pytest.mark.parametrize("K,g,layered", [(2, 0.0, False), (3, 0.05, False), (4, 0.0, False), (3, 0.0, True)])
def test_retro_chain_batch_equals_single_pings(K, g, layered):
    """A batch with retro-chain returns (mixed layouts and poses, one
    persistent launch) writes the same volumes, bit for bit, as single pings."""
    torch, sonar = _gpu()
    sc = sonar.Scene(_surface_wall())
    base = _cfg(max_bounces=K, c_grad=g, ssp=KNOTS if layered else ())
    items = [(base.replace(n_h=nh, n_v=nv, rays_per_beam=nr),
              S.pose((0.3 * i, -0.2 * i, -0.5 * i), pitch_down=math.radians(-10 + 3 * i), ping=i))
             for i, (nh, nv, nr) in enumerate([(32, 16, 4), (16, 8, 16), (33, 7, 1), (64, 32, 4)])]
    b = sonar.Batch(sc, items)
    assert b.plan.retro == 1
    b.run()
    torch.cuda.synchronize()
    assert sc.status() == 0
    for i, (cfg, pose) in enumerate(items):
        ref = sonar.ping(sc, cfg, pose)["volume"]
        torch.cuda.synchronize()
        assert torch.equal(b.volumes[i].view(torch.float32), ref.view(torch.float32)), i
