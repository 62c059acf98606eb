"""Monte-Carlo continuation (directions drawn from the Lambert and Phong
lobes by a counter-based generator) on the GPU against the FP64 oracle,
through the C-ABI (needs an MI355X)."""
import math

import numpy as np
import pytest

from paper_2606_06130_amd import scenes as S
from tests import meshes as M
from tests.test_gpu_parity import _gpu, assert_parity, run_parity

pytestmark = pytest.mark.gpu

DIFFUSE = 4


def _surface_boxes():
    surface = M.mesh_from([M.big_triangle_z(1.0)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    mesh = M.concat(S.scene_seabed_boxes(), surface)
    mesh.name = "boxes_surface"
    return mesh


@pytest.mark.parametrize("K,g,seed", [(2, 0.0, 1), (3, 0.0, 77), (3, 0.05, 5), (4, 0.0, 9)])
def test_seabed_boxes_under_a_surface_drawn_continuations(K, g, seed):
    cfg = S.sensor_seabed_boxes().replace(n_h=16, n_v=8, rays_per_beam=4, n_range=512, max_bounces=K, k_d=0.7,
                                          k_s=0.3, phong_n=20.0, c_grad=g, seed=seed, flags=DIFFUSE)
    res, g_, orc = run_parity(_surface_boxes(), cfg, S.pose_seabed_boxes())
    assert_parity(res, K)
    assert (orc["tri"][:, 1] >= 0).sum() > 20          # drawn paths reach further facets


def test_batch_with_drawn_continuations_equals_single_pings():
    torch, sonar = _gpu()
    mesh = _surface_boxes()
    sc = sonar.Scene(mesh)
    base = S.sensor_seabed_boxes().replace(max_bounces=3, k_d=0.7, k_s=0.3, flags=DIFFUSE)
    items = [(base.replace(n_h=nh, n_v=nv, rays_per_beam=nr), S.pose((0.1 * i, 0.0, 0.0), pitch_down=math.radians(55),
                                                                     ping=i))
             for i, (nh, nv, nr) in enumerate([(8, 4, 4), (16, 8, 16), (33, 7, 1)])]
    b = sonar.Batch(sc, items)
    b.run()
    torch.cuda.synchronize()
    for i, (cfg, pose) in enumerate(items):
        ref = sonar.ping(sc, cfg, pose)["volume"]
        torch.cuda.synchronize()
        assert torch.equal(b.volumes[i].view(torch.float32), ref.view(torch.float32))
