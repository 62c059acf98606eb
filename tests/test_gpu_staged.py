"""The staged multi-bounce ping (one kernel per traversal kind, FP64 ray
state through a workspace) against the fused single kernel and against the
oracle (needs an MI355X)."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2606_06130_amd import scenes as S
from tests import meshes as M
from tests.parity import compare_rays, mask_words, ray_ids, rel_l2

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU (it must not pass by skipping)")
    from paper_2606_06130_amd import sonar
    return torch, sonar


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _surface_wall():
    surf = M.mesh_from([M.big_triangle_z(2.0)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    rng = np.random.Generator(np.random.PCG64(1))
    wall = M.plane_grid_x(8.0, -6.0, 6.0, -8.0, 2.0, 40, rng)
    mesh = M.concat(surf, wall)
    mesh.name = "surface_wall"
    return mesh


CASES = {
    "boxes_straight_k3": lambda sonar: (S.scene_seabed_boxes(),
                                        S.sensor_seabed_boxes().replace(max_bounces=3, k_d=0.7, k_s=0.3, n_range=512),
                                        S.pose_seabed_boxes()),
    "boxes_gradient_k2": lambda sonar: (S.scene_seabed_boxes(),
                                        S.sensor_seabed_boxes().replace(max_bounces=2, k_d=0.7, k_s=0.3, n_range=777,
                                                                        c_grad=0.05), S.pose_seabed_boxes()),
    "surface_wall_k4_gradient": lambda sonar: (_surface_wall(),
                                               S.SensorConfig(n_h=32, n_v=16, rays_per_beam=4, n_range=1024,
                                                              max_bounces=4, k_d=0.7, k_s=0.3,
                                                              vfov=math.radians(60), c_grad=0.05),
                                               S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10))),
    "surface_wall_retro_pattern": lambda sonar: (_surface_wall(),
                                                 S.SensorConfig(n_h=32, n_v=16, rays_per_beam=8, n_range=1024,
                                                                max_bounces=3, k_d=0.7, k_s=0.3,
                                                                vfov=math.radians(60),
                                                                flags=sonar.FLAG_RETRO_CHAIN | sonar.FLAG_BEAM_PATTERN),
                                                 S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10))),
    "surface_wall_diffuse": lambda sonar: (_surface_wall(),
                                           S.SensorConfig(n_h=33, n_v=7, rays_per_beam=16, n_range=600,
                                                          max_bounces=3, k_d=0.7, k_s=0.3,
                                                          vfov=math.radians(60), c_grad=-0.08,
                                                          flags=sonar.FLAG_DIFFUSE_BOUNCE),
                                           S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10))),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_staged_equals_fused(case):
    """Records bit-exact; volume, G-buffer and incoherent channels equal up
    to FP32 rounding (the same arithmetic in other kernels)."""
    torch, sonar = _gpu()
    mesh, cfg, pose = CASES[case](sonar)
    sc = sonar.Scene(mesh)
    a = sonar.ping(sc, cfg, pose, gbuffer=True, incoh=True, record=True)
    b = sonar.ping(sc, cfg, pose, gbuffer=True, incoh=True, record=True, staged=True)
    torch.cuda.synchronize()
    assert sc.status() == 0
    for k in ("tri", "bin", "vis", "beam", "rbin"):
        if k in a:
            assert torch.equal(a[k], b[k]), (case, k)
    for k in ("amp", "ramp", "volume", "incoh"):
        if k in a:
            x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
            assert rel_l2(y, x) <= 1e-6, (case, k, rel_l2(y, x))
    assert np.abs(a["gbuffer"].cpu().numpy() - b["gbuffer"].cpu().numpy()).max() <= 1e-6
    same = torch.equal(a["volume"].view(torch.float32), b["volume"].view(torch.float32))
    _log(case, "volume bit-identical to the fused kernel:", same)


def test_staged_receive_binning_equals_fused():
    """Receive binning with several bounces: the list of moved returns comes
    from the accumulation stage (atomics place them: volumes to rounding)."""
    torch, sonar = _gpu()
    mesh = _surface_wall()
    cfg = S.SensorConfig(n_h=32, n_v=16, rays_per_beam=4, n_range=1024, max_bounces=3, k_d=0.7, k_s=0.3,
                         vfov=math.radians(60), c_grad=0.05, flags=sonar.FLAG_RX_BEAMS | sonar.FLAG_BEAM_PATTERN)
    pose = S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10))
    sc = sonar.Scene(mesh)
    a = sonar.ping(sc, cfg, pose, incoh=True, record=True)
    b = sonar.ping(sc, cfg, pose, incoh=True, record=True, staged=True)
    torch.cuda.synchronize()
    for k in ("tri", "bin", "vis", "beam"):
        assert torch.equal(a[k], b[k]), k
    assert rel_l2(b["volume"].cpu().numpy(), a["volume"].cpu().numpy()) <= 1e-6
    assert rel_l2(b["incoh"].cpu().numpy(), a["incoh"].cpu().numpy()) <= 1e-6


def test_staged_harbor_multipath_every_ray_matches_oracle():
    """The full 1,991,680-triangle multipath ping through the staged kernels,
    every ray against the oracle (flagged rays masked on both sides)."""
    torch, sonar = _gpu()
    mesh = S.scene_harbor_multipath()
    cfg, pose = S.sensor_harbor_multipath(), S.pose_harbor()
    orc = oracle.trace_beams(oracle.Scene(mesh), cfg, pose, np.arange(cfg.n_beams), want_incoh=True, want_gbuf=True)
    rays = ray_ids(np.arange(cfg.n_beams), cfg.rays_per_beam)
    mask = torch.from_numpy(mask_words(cfg.n_rays, rays[orc["flags"] != 0])).cuda()
    sc = sonar.Scene(mesh)
    out = sonar.ping(sc, cfg, pose, gbuffer=True, incoh=True, record=True, ray_mask=mask, staged=True)
    torch.cuda.synchronize()
    assert sc.status() == 0
    g = {k: v.cpu().numpy() for k, v in out.items() if k != "workspace"}
    res = compare_rays(g, orc, rays)
    _log("staged multipath", res)
    for key in ("tri_mismatch", "bin_mismatch", "vis_mismatch"):
        assert res[key] == 0, res
    ok = orc["flags"] == 0
    assert rel_l2(g["amp"][ok], orc["amp"][ok]) <= 1e-4
    nb = cfg.n_beams
    assert rel_l2(g["volume"].reshape(nb, -1), orc["col"]) <= 1e-4
    inc = g["incoh"].reshape(2, nb, -1)
    assert rel_l2(inc[0], orc["incoh"][:, 0]) <= 1e-4
    assert rel_l2(inc[1], orc["incoh"][:, 1]) <= 1e-4
    assert np.abs(g["gbuffer"].reshape(nb, 8) - orc["gbuf"]).max() <= 1e-5
    assert res["flagged"] <= 0.01 * 5 * res["rays"]


def test_staged_workspace_validation():
    torch, sonar = _gpu()
    import ctypes as C
    sc = sonar.Scene(S.scene_seabed_boxes())
    cfg = S.sensor_seabed_boxes().replace(max_bounces=3, k_d=0.7, k_s=0.3)
    p = sonar.params_of(cfg)
    need = sonar.lib().sonar_workspace_size(sc.handle, C.byref(p), 1)
    assert need >= cfg.n_rays * (80 + 64 + 3 * 20)
    assert sonar.lib().sonar_workspace_size(sc.handle, C.byref(p), 3) == 3 * need
    p1 = sonar.params_of(cfg.replace(max_bounces=1))
    assert sonar.lib().sonar_workspace_size(sc.handle, C.byref(p1), 1) == 0
    out = sonar.alloc_outputs(cfg)
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    q = sonar.pose_of(S.pose_seabed_boxes())
    st = sonar.lib().sonar_ping_ws(sc.handle, C.byref(p), C.byref(q), out["volume"].data_ptr(), None, None, None,
                                   None, ws.data_ptr(), ws.numel(), None)
    assert st == sonar.SONAR_E_INVALID
