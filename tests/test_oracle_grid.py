"""The oracle's uniform-grid candidate filter is exact: with it, traces are
bit-identical to the brute-force loop over every triangle (indices, flags,
contributions, columns, G-buffer, incoherent channels), on the benchmark
scenes and on small scenes with the grid forced at several cell sizes, over
every path option (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from paper_2606_06130_amd import scenes as S
from tests import meshes as M


def _same(a, b):
    for k in a:
        x, y = a[k], b[k]
        if x.dtype.kind == "c":
            x, y = x.view(np.float64), y.view(np.float64)
        assert np.array_equal(x, y), k


def _trace(sc, cfg, pose, beams):
    return oracle.trace_beams(sc, cfg, pose, beams, want_incoh=True, want_gbuf=True)


def test_grid_harbor_single_bounce_4096_rays():
    mesh = S.scene_harbor()
    cfg, pose = S.sensor_harbor(), S.pose_harbor()
    g, b = oracle.Scene(mesh), oracle.Scene(mesh, grid=False)
    assert g.grid_info()["cells"] > 0 and b.grid_info()["cells"] == 0
    beams = np.sort(np.random.Generator(np.random.PCG64(5)).choice(cfg.n_beams, 256, replace=False))
    rg = _trace(g, cfg, pose, beams)
    assert (rg["tri"] >= 0).mean() > 0.9
    _same(rg, _trace(b, cfg, pose, beams))


def test_grid_harbor_multipath_sampled_rays():
    """1.99M triangles, 3 bounces in c(z) = 1500 + 0.05 z: arcs, eigenray
    connections and their visibility queries."""
    mesh = S.scene_harbor_multipath()
    cfg, pose = S.sensor_harbor_multipath(), S.pose_harbor()
    g, b = oracle.Scene(mesh), oracle.Scene(mesh, grid=False)
    beams = np.sort(np.random.Generator(np.random.PCG64(6)).choice(cfg.n_beams, 12, replace=False))
    rg = _trace(g, cfg, pose, beams)
    assert (rg["tri"][:, 1] >= 0).any() and (rg["vis"][:, 1] == 1).any()
    _same(rg, _trace(b, cfg, pose, beams))


@pytest.mark.parametrize("cells_per_triangle", [0.05, 0.5, 8.0])
@pytest.mark.parametrize("case", ["boxes_gradient", "boxes_layered_retro", "surface_wall_rx_diffuse"])
def test_grid_forced_small_scenes(case, cells_per_triangle):
    if case.startswith("boxes"):
        mesh = S.scene_seabed_boxes()
        cfg = S.sensor_seabed_boxes().replace(n_h=32, n_v=16, max_bounces=3, k_d=0.7, k_s=0.3, n_range=512)
        pose = S.pose_seabed_boxes()
        if case == "boxes_gradient":
            cfg = cfg.replace(c_grad=0.05)
        else:
            cfg = cfg.replace(ssp=((-9.0, 1499.6), (-4.0, 1500.3), (-1.0, 1499.9), (1.5, 1500.2)),
                              flags=oracle.RETRO_CHAIN)
    else:
        surf = M.mesh_from([M.big_triangle_z(2.0)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
        rng = np.random.Generator(np.random.PCG64(1))
        wall = M.plane_grid_x(8.0, -6.0, 6.0, -8.0, 2.0, 40, rng)
        mesh = M.concat(surf, wall)
        cfg = S.SensorConfig(n_h=32, n_v=16, rays_per_beam=4, n_range=1024, max_bounces=4, k_d=0.7, k_s=0.3,
                             vfov=math.radians(60), c_grad=0.05,
                             flags=oracle.RX_BEAMS | oracle.BEAM_PATTERN | oracle.DIFFUSE_BOUNCE)
        pose = S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10))
    g = oracle.Scene(mesh, grid=True, cells_per_triangle=cells_per_triangle)
    b = oracle.Scene(mesh, grid=False)
    beams = np.arange(cfg.n_beams)
    rg = _trace(g, cfg, pose, beams)
    assert (rg["tri"] >= 0).sum() > 0
    _same(rg, _trace(b, cfg, pose, beams))


def test_grid_forced_slivers_and_deep_chain():
    """Clusters of identical slivers (large grown boxes) and a wall."""
    mesh = M.deep_chain()
    cfg = S.SensorConfig(n_h=16, n_v=8, rays_per_beam=4, n_range=512, hfov=math.radians(10.0),
                         vfov=math.radians(10.0), max_bounces=2, k_d=0.7, k_s=0.3)
    pose = S.pose((3.0, 0.0, 0.0), yaw=math.pi)
    g, b = oracle.Scene(mesh, grid=True, cells_per_triangle=4.0), oracle.Scene(mesh, grid=False)
    beams = np.arange(cfg.n_beams)
    _same(_trace(g, cfg, pose, beams), _trace(b, cfg, pose, beams))
