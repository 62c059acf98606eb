"""HIP path vs FP64 oracle, through the C-ABI (needs an MI355X)."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2606_06130_amd import scenes as S
from tests import meshes as M
from tests.parity import compare_points as _compare_points, compare_rays, mask_words, ray_ids, rel_l2

pytestmark = pytest.mark.gpu

VOL_TOL = 1e-4          # relative L2 of the echo volume, flagged rays masked on both sides


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU (it must not pass by skipping)")
    from paper_2606_06130_amd import sonar
    return torch, sonar


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_parity(mesh, cfg, pose, beams=None, gbuffer=True, incoh=True, orc_scene=None, gpu_scene=None):
    """Full ping on the GPU with the oracle's flagged rays masked; the oracle
    traces the listed beams (all by default). Returns a dict of measures."""
    torch, sonar = _gpu()
    nb = cfg.n_beams
    beams = np.arange(nb) if beams is None else np.asarray(beams)
    osc = orc_scene or oracle.Scene(mesh)
    orc = oracle.trace_beams(osc, cfg, pose, beams, want_incoh=incoh, want_gbuf=gbuffer)
    rays = ray_ids(beams, cfg.rays_per_beam)
    flagged = rays[orc["flags"] != 0]
    mask = torch.from_numpy(mask_words(nb * cfg.rays_per_beam, flagged)).cuda()
    sc = gpu_scene or sonar.Scene(mesh)
    out = sonar.ping(sc, cfg, pose, gbuffer=gbuffer, incoh=incoh, record=True, ray_mask=mask)
    torch.cuda.synchronize()
    assert sc.status() == 0
    g = {k: v.cpu().numpy() for k, v in out.items()}
    res = compare_rays(g, orc, rays)
    res["bounces"] = cfg.max_bounces
    vol = g["volume"].reshape(nb, cfg.n_range)[beams]
    res["vol_err"] = rel_l2(vol, orc["col"])
    res["vol_err_unmasked_vs_all"] = None
    res["energy"] = float((np.abs(orc["col"]) ** 2).sum())
    if incoh:
        inc = g["incoh"].reshape(2, nb, cfg.n_range)[:, beams]
        res["i1_err"] = rel_l2(inc[0], orc["incoh"][:, 0])
        res["im_err"] = rel_l2(inc[1], orc["incoh"][:, 1])
        res["im_energy"] = float(orc["incoh"][:, 1].sum())
    if gbuffer:
        gb = g["gbuffer"].reshape(nb, 8)[beams]
        res["gbuf_err"] = float(np.abs(gb - orc["gbuf"]).max())
    res["contrib_err"] = 0.0
    ok = orc["flags"] == 0
    ga = g["amp"][rays][ok]
    oa = orc["amp"][ok]
    if np.abs(oa).sum() > 0:
        res["contrib_err"] = rel_l2(ga, oa)
    _log(mesh.name, cfg.n_h, cfg.n_v, cfg.rays_per_beam, cfg.n_range, cfg.max_bounces, res)
    return res, g, orc


def assert_parity(res, bounces=1):
    assert res["tri_mismatch"] == 0, res
    assert res["bin_mismatch"] == 0, res
    assert res["vis_mismatch"] == 0, res
    assert res.get("beam_mismatch", 0) == 0, res
    assert res.get("rbin_mismatch", 0) == 0, res
    assert res.get("retro_err", 0.0) <= VOL_TOL, res
    assert res["vol_err"] <= VOL_TOL, res
    assert res["contrib_err"] <= VOL_TOL, res
    if "i1_err" in res:
        assert res["i1_err"] <= VOL_TOL, res
        if res.get("im_energy", 0) > 0:
            assert res["im_err"] <= VOL_TOL, res
    if "gbuf_err" in res:
        assert res["gbuf_err"] <= 1e-5, res
    # at most 1% of the traversals (K nearest-hit + K - 1 connection queries per ray) flagged
    assert res["flagged"] <= max(0.01 * (2 * res.get("bounces", 1) - 1) * res["rays"], 2), res


# ---------------------------------------------------------------------------


def test_seabed_boxes_single_bounce_full():
    """2,128 triangles, 64 x 32 beams x 4 rays, 256 bins: every ray compared."""
    mesh = S.scene_seabed_boxes()
    res, g, orc = run_parity(mesh, S.sensor_seabed_boxes(), S.pose_seabed_boxes())
    assert_parity(res)
    assert res["energy"] > 0


def test_seabed_boxes_deterministic():
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    cfg, pose = S.sensor_seabed_boxes(), S.pose_seabed_boxes()
    sc = sonar.Scene(mesh)
    a = sonar.ping(sc, cfg, pose, incoh=True)["volume"].clone()
    b = sonar.ping(sc, cfg, pose, incoh=True)["volume"].clone()
    sc2 = sonar.Scene(mesh)
    c = sonar.ping(sc2, cfg, pose)["volume"]
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.float32), b.view(torch.float32))
    assert torch.equal(a.view(torch.float32), c.view(torch.float32))


def test_level_pose_volume_is_empty():
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    sc = sonar.Scene(mesh)
    out = sonar.alloc_outputs(S.sensor_seabed_boxes())
    out["volume"].fill_(1.0)
    sonar.ping(sc, S.sensor_seabed_boxes(), S.pose_seabed_boxes_level(), out=out)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(out["volume"])) == 0


@pytest.mark.parametrize("n_h,n_v,n_r,n_range,mode", [
    (7, 5, 4, 257, 0),        # ragged: 140 rays, odd bin count
    (13, 11, 1, 200, 0),      # one ray per beam
    (9, 3, 64, 128, 0),       # one beam per wave
    (10, 6, 1, 300, 1),       # LiDAR firing grid: 11 x 7 emitters
    (33, 17, 2, 64, 0),
])
def test_seabed_boxes_layouts(n_h, n_v, n_r, n_range, mode):
    mesh = S.scene_seabed_boxes()
    cfg = S.sensor_seabed_boxes().replace(n_h=n_h, n_v=n_v, rays_per_beam=n_r, n_range=n_range, grid_mode=mode,
                                          jitter=0 if mode == 1 else 1)
    # a slight yaw keeps the LiDAR grid's exact lattice angles off the seabed's exact lattice edges
    pose = S.pose((0.0, 0.0, 0.0), yaw=0.0123, pitch_down=math.radians(60.0))
    res, _, _ = run_parity(mesh, cfg, pose)
    assert_parity(res)


def test_single_triangle_scene():
    mesh = M.mesh_from([M.big_triangle_x(6.0)], rho=0.3, phi=0.2)
    mesh.name = "one_triangle"
    cfg = S.SensorConfig(n_h=16, n_v=8, rays_per_beam=4, n_range=512)
    res, _, _ = run_parity(mesh, cfg, S.pose((0.0, 0.0, 0.0)))
    assert_parity(res)


def test_multibounce_straight_seabed_boxes():
    mesh = S.scene_seabed_boxes()
    cfg = S.sensor_seabed_boxes().replace(max_bounces=3, k_d=0.7, k_s=0.3, n_range=512)
    res, _, _ = run_parity(mesh, cfg, S.pose_seabed_boxes())
    assert_parity(res)


def test_surface_multipath_straight():
    """Pressure-release surface + wall, 2 bounces, constant c."""
    surf = M.mesh_from([M.big_triangle_z(2.0)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    rng = np.random.Generator(np.random.PCG64(1))
    wall = M.plane_grid_x(8.0, -6.0, 6.0, -8.0, 2.0, 40, rng)
    mesh = M.concat(surf, wall)
    mesh.name = "surface_wall"
    cfg = S.SensorConfig(n_h=32, n_v=16, rays_per_beam=4, n_range=1024, max_bounces=3, k_d=0.7, k_s=0.3,
                         vfov=math.radians(60))
    res, _, _ = run_parity(mesh, cfg, S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10)))
    assert_parity(res)
    assert res["im_energy"] > 0


def test_harbor_full_size_every_ray():
    """601,088 triangles, 256 x 128 beams x 16 rays, 1,024 bins: the full ping
    as benchmarked, every one of its 524,288 rays compared with the oracle ray
    by ray and every beam column by column (volume, G-buffer, incoherent
    channel)."""
    mesh = S.scene_harbor()
    cfg, pose = S.sensor_harbor(), S.pose_harbor()
    res, g, orc = run_parity(mesh, cfg, pose)
    assert_parity(res)
    assert res["rays"] == cfg.n_rays


@pytest.mark.parametrize("n_range,train,guard,M", [
    (1, 16, 4, 4), (2, 1, 0, 1), (3, 2, 0, 2), (77, 8, 2, 4), (256, 16, 4, 16), (1000, 16, 4, 4),
    (4096, 64, 8, 16)])
def test_detect_synthetic_volumes_match_oracle(n_range, train, guard, M):
    """CFAR on seeded sparse volumes (log-normal returns with random phase,
    two-bin plateaus, Rayleigh-noise beams) over every per-lane chunk size and
    both load paths (odd and even bin counts), all beams against the oracle."""
    torch, sonar = _gpu()
    cfg = S.SensorConfig(n_h=8, n_v=8, rays_per_beam=1, jitter=0, n_range=n_range)
    pose = S.pose((1.0, -2.0, -3.0), yaw=0.3, pitch_down=0.4)
    rng = np.random.Generator(np.random.PCG64(100 + n_range))
    nb = cfg.n_beams
    v = np.zeros((nb, n_range), np.complex64)
    for b in range(nb):
        if b % 8 == 7:
            v[b] = (rng.normal(size=n_range) + 1j * rng.normal(size=n_range)) * np.sqrt(5e-11)
            continue
        k = int(rng.integers(0, n_range // 8 + 2))
        bins = rng.choice(n_range, min(k, n_range), replace=False)
        v[b, bins] = np.exp(rng.normal(-9.0, 3.0, len(bins))) * np.exp(2j * np.pi * rng.random(len(bins)))
        if n_range >= 4 and b % 8 == 3:
            r = int(rng.integers(1, n_range - 2))
            v[b, r] = v[b, r + 1] = 1e-3
    det = sonar.Detector(cfg, train=train, guard=guard, max_per_beam=M)
    det(torch.from_numpy(v).cuda(), pose)
    pts, total = det.fetch()
    o = oracle.detect(v, cfg, pose, np.arange(nb), train=train, guard=guard, max_per_beam=M)
    compared = _compare_points(pts, total, o, np.arange(nb))
    _log("synthetic CFAR", n_range, "points", total, "beams compared", compared)
    assert compared >= 0.75 * nb
    if n_range >= 77:
        assert total > 0


def test_harbor_cfar_points_match_oracle():
    """Detection on the same FP32 volume: identical point sets except
    decisions within 1e-4 of their threshold."""
    torch, sonar = _gpu()
    mesh = S.scene_harbor()
    cfg, pose = S.sensor_harbor(), S.pose_harbor()
    sc = sonar.Scene(mesh)
    vol = sonar.ping(sc, cfg, pose)["volume"]
    det = sonar.Detector(cfg)
    det(vol, pose)
    pts, total = det.fetch()
    v = vol.cpu().numpy().reshape(cfg.n_beams, cfg.n_range)
    rng = np.random.Generator(np.random.PCG64(9))
    beams = np.sort(rng.choice(cfg.n_beams, 2048, replace=False))
    o = oracle.detect(v, cfg, pose, beams)
    compared = _compare_points(pts, total, o, beams)
    assert compared > 1900
    assert total > 0


def test_detect_capacity_truncates():
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    cfg, pose = S.sensor_seabed_boxes(), S.pose_seabed_boxes()
    sc = sonar.Scene(mesh)
    vol = sonar.ping(sc, cfg, pose)["volume"]
    full = sonar.Detector(cfg)
    full(vol, pose)
    p_full, n_full = full.fetch()
    assert n_full > 10
    small = sonar.Detector(cfg, capacity=5)
    small(vol, pose)
    p_small, n_small = small.fetch()
    assert n_small == n_full
    assert len(p_small) == 5
    assert np.array_equal(p_small.view(np.int32), p_full[:5].view(np.int32))


def test_build_rejects_bad_index():
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    bad = S.Mesh(mesh.vertices, mesh.indices.copy(), mesh.reflectivity, mesh.phase, mesh.material)
    bad.indices[5, 1] = mesh.vertices.shape[0]
    with pytest.raises(sonar.SonarError) as e:
        sonar.Scene(bad)
    assert e.value.status == sonar.SONAR_E_INVALID


def test_build_rejects_nan_vertex():
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    v = mesh.vertices.copy()
    v[3, 2] = np.nan
    with pytest.raises(sonar.SonarError):
        sonar.Scene(S.Mesh(v, mesh.indices, mesh.reflectivity, mesh.phase, mesh.material))


def test_scene_info_and_device_inputs():
    torch, sonar = _gpu()
    mesh = S.scene_harbor()
    a = sonar.Scene(mesh)
    b = sonar.Scene(mesh, device_inputs=True)
    ia, ib = a.info(), b.info()
    assert ia == ib
    assert ia["n_triangles"] == mesh.n_triangles
    np.testing.assert_allclose(ia["lo"], mesh.vertices.min(0))
    np.testing.assert_allclose(ia["hi"], mesh.vertices.max(0))
    assert 1 <= ia["depth"] <= 64
    _log("harbor hierarchy", ia)


def _scene_of(which):
    if which == "harbor":
        return S.scene_harbor(), S.sensor_harbor(), S.pose_harbor()
    return S.scene_seabed_boxes(), S.sensor_seabed_boxes(), S.pose_seabed_boxes()


def _by_beam(pts):
    out = {}
    for p in pts:
        out.setdefault(int(p["beam"]), []).append(int(p["bin"]))
    return out


@pytest.mark.parametrize("which", ["harbor", "boxes"])
def test_fused_ping_detect_matches_separate(which):
    """sonar_ping_detect == sonar_ping + sonar_detect: same volume bits; the
    point lists of a beam differ only where a decision of the beam lies within
    1e-6 relative of its CFAR threshold or of a neighbour's power (FP32
    rounding of the power, FP64 order of the training sums), or the top-M
    choice is that close: every differing beam is checked against the
    oracle's flags computed from the shared volume."""
    torch, sonar = _gpu()
    mesh, cfg, pose = _scene_of(which)
    sc = sonar.Scene(mesh)
    v1 = sonar.ping(sc, cfg, pose)["volume"]
    d1 = sonar.Detector(cfg)
    d1(v1, pose)
    p1, n1 = d1.fetch()
    v2 = torch.empty_like(v1)
    d2 = sonar.Detector(cfg)
    d2.ping_detect(sc, v2, pose)
    p2, n2 = d2.fetch()
    assert torch.equal(v1.view(torch.float32), v2.view(torch.float32))
    assert n1 > 0
    b1, b2 = _by_beam(p1), _by_beam(p2)
    differ = sorted(b for b in set(b1) | set(b2) if b1.get(b, []) != b2.get(b, []))
    _log(which, "detections", n1, n2, "beams that differ", len(differ))
    if differ:
        v = v1.cpu().numpy().reshape(cfg.n_beams, cfg.n_range)
        o = oracle.detect(v, cfg, pose, np.array(differ), rel_thr=1e-6, rel_peak=1e-6)
        for q, b in enumerate(differ):
            bins = set(b1.get(b, [])) ^ set(b2.get(b, []))
            assert o["beam_flag"][q] or any(o["flag_bins"][q][x] for x in bins) or \
                set(b1.get(b, [])) == set(b2.get(b, [])), (b, b1.get(b), b2.get(b))
    common = sorted(set(zip(p1["beam"].tolist(), p1["bin"].tolist())) & set(zip(p2["beam"].tolist(),
                                                                                 p2["bin"].tolist())))
    i1 = {k: i for i, k in enumerate(zip(p1["beam"].tolist(), p1["bin"].tolist()))}
    i2 = {k: i for i, k in enumerate(zip(p2["beam"].tolist(), p2["bin"].tolist()))}
    a = p1[[i1[k] for k in common]]
    b = p2[[i2[k] for k in common]]
    for f in ("x", "y", "z"):
        np.testing.assert_array_equal(a[f], b[f])
    # the FP32 power may differ in its last bit (fused multiply-add contraction)
    np.testing.assert_allclose(a["db"], b["db"], rtol=1e-6)


@pytest.mark.parametrize("which", ["harbor", "boxes"])
def test_fused_ping_detect_matches_oracle(which):
    """The fused call's points against the oracle's detection on the fused
    call's own volume, every beam: identical bins, positions and powers on
    every beam without a flagged decision (within 1e-4 of a threshold or 1e-6
    of a neighbour); flagged beams are counted."""
    torch, sonar = _gpu()
    mesh, cfg, pose = _scene_of(which)
    sc = sonar.Scene(mesh)
    vol = torch.empty(sonar.beams_of(cfg) + (cfg.n_range,), dtype=torch.complex64, device="cuda")
    det = sonar.Detector(cfg)
    det.ping_detect(sc, vol, pose)
    pts, total = det.fetch()
    v = vol.cpu().numpy().reshape(cfg.n_beams, cfg.n_range)
    beams = np.arange(cfg.n_beams)
    o = oracle.detect(v, cfg, pose, beams)
    compared = _compare_points(pts, total, o, beams)
    skipped = cfg.n_beams - compared
    _log(which, "fused CFAR vs oracle: points", total, "beams compared", compared, "flagged beams", skipped)
    assert total > 0
    assert skipped <= max(0.01 * cfg.n_beams, 2)


# ---------------------------------------------------------------------------
# curved rays: c(z) = c0 + g z


@pytest.mark.parametrize("g", [0.05, -0.08])
def test_seabed_boxes_gradient_single_bounce(g):
    mesh = S.scene_seabed_boxes()
    cfg = S.sensor_seabed_boxes().replace(c_grad=g)
    res, _, _ = run_parity(mesh, cfg, S.pose_seabed_boxes())
    assert_parity(res)


def test_surface_multipath_gradient():
    """Pressure-release surface + wall in c(z) = 1500 + 0.05 z, 3 bounces:
    curved first legs and eigenray connections with visibility."""
    surf = M.mesh_from([M.big_triangle_z(2.0)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    rng = np.random.Generator(np.random.PCG64(1))
    wall = M.plane_grid_x(8.0, -6.0, 6.0, -8.0, 2.0, 40, rng)
    mesh = M.concat(surf, wall)
    mesh.name = "surface_wall_gradient"
    cfg = S.SensorConfig(n_h=32, n_v=16, rays_per_beam=4, n_range=1024, max_bounces=3, k_d=0.7, k_s=0.3,
                         vfov=math.radians(60), c_grad=0.05)
    res, _, _ = run_parity(mesh, cfg, S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10)))
    assert_parity(res)
    assert res["im_energy"] > 0


def test_multibounce_gradient_seabed_boxes():
    mesh = S.scene_seabed_boxes()
    cfg = S.sensor_seabed_boxes().replace(max_bounces=3, k_d=0.7, k_s=0.3, n_range=1024, c_grad=0.05)
    res, _, _ = run_parity(mesh, cfg, S.pose_seabed_boxes())
    assert_parity(res)


def test_harbor_multipath_full_size_every_ray():
    """1,991,680 triangles (wall, seabed, surface, 50 piles), 3 bounces, Phong-20
    + diffuse, c(z) = 1500 + 0.05 z, 256 x 128 beams x 16 rays, 1,024 bins: the
    full ping, every ray compared bounce by bounce and every beam column by
    column."""
    mesh = S.scene_harbor_multipath()
    cfg, pose = S.sensor_harbor_multipath(), S.pose_harbor()
    res, g, orc = run_parity(mesh, cfg, pose)
    assert_parity(res, bounces=3)
    assert res["rays"] == cfg.n_rays
    assert res["im_energy"] > 0


def test_deep_hierarchy_stack_spills_past_lds():
    """A chain hierarchy whose traversals need more stack entries than the
    single-bounce LDS stack holds: the deeper entries live in private memory,
    and every ray still matches the oracle."""
    torch, sonar = _gpu()
    mesh = M.deep_chain()
    mesh.name = "deep_chain"
    cfg = S.SensorConfig(n_h=16, n_v=8, rays_per_beam=4, n_range=512, hfov=math.radians(10.0),
                         vfov=math.radians(10.0))
    pose = S.pose((3.0, 0.0, 0.0), yaw=math.pi)
    sc = sonar.Scene(mesh)
    depth = sc.info()["depth"]          # levels of 4-wide nodes: three pushes each at most
    assert 3 * depth > 20 and 3 * depth <= 64, depth
    st = sonar.ping(sc, cfg, pose, record=True, stats=True)
    torch.cuda.synchronize()
    deepest = int(st["stats"][:, 2].max().item())
    _log("deep chain: hierarchy depth", depth, "deepest stack", deepest)
    assert deepest > 20
    res, g, _ = run_parity(mesh, cfg, pose, gpu_scene=sc)
    assert_parity(res)
    assert res["energy"] > 0
    assert (g["tri"][:, 0] == mesh.indices.shape[0] - 1).all()     # every ray reaches the wall


@pytest.mark.parametrize("bounces,g", [(1, 0.0), (3, 0.05)])
def test_traversal_counters_keep_results(bounces, g):
    """The counting kernels return the same indices and bins as the plain
    ones, values equal up to rounding, and plausible counts."""
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    cfg = S.sensor_seabed_boxes().replace(max_bounces=bounces, k_d=0.7, k_s=0.3, c_grad=g)
    pose = S.pose_seabed_boxes()
    sc = sonar.Scene(mesh)
    a = sonar.ping(sc, cfg, pose, record=True, stats=True)
    b = sonar.ping(sc, cfg, pose, record=True)
    torch.cuda.synchronize()
    assert sc.status() == 0
    for k in ("tri", "bin", "vis"):
        assert torch.equal(a[k], b[k]), k
    va, vb = a["volume"].cpu().numpy(), b["volume"].cpu().numpy()
    assert rel_l2(va, vb) <= 1e-9
    st = a["stats"].cpu().numpy()
    tri = a["tri"].cpu().numpy()
    assert (st[:, 0] >= 1).all()                      # the root is an internal node
    assert (st[tri[:, 0] >= 0, 1] >= 1).all()         # a hit needs a tested triangle
    assert (st[:, 2] <= 3 * sc.info()["depth"]).all()     # at most three pushes per level of 4-wide nodes


@pytest.mark.parametrize("n_tri,leaf", [(2, 0), (3, 0), (4, 0), (5, 0), (5, 1), (9, 2), (17, 8)])
def test_tiny_scenes(n_tri, leaf):
    """Scenes of a few triangles: a single 4-wide node with one leaf (at most
    leaf_size triangles), sparse nodes with empty child slots, leaf sizes 1-8;
    overlapping triangles at staggered depths so nearer ones occlude."""
    torch, sonar = _gpu()
    tris = []
    for k in range(n_tri):
        a = 2.0 * math.pi * k / n_tri
        y0, z0, x = 0.6 * math.cos(a), 0.6 * math.sin(a), 5.0 + 0.35 * k
        tris.append([[x, y0 - 0.9, z0 - 0.7], [x + 0.2, y0 + 0.9, z0 - 0.6], [x - 0.1, y0 + 0.1, z0 + 0.9]])
    mesh = M.mesh_from(tris, rho=0.4, phi=0.3)
    mesh.name = f"tiny{n_tri}"
    cfg = S.SensorConfig(n_h=16, n_v=8, rays_per_beam=4, n_range=512, hfov=math.radians(40.0),
                         vfov=math.radians(30.0))
    sc = sonar.Scene(mesh, leaf_size=leaf)
    info = sc.info()
    assert info["n_triangles"] == n_tri and info["n_nodes"] >= 1
    res, g, _ = run_parity(mesh, cfg, S.pose((0.0, 0.0, 0.0)), gpu_scene=sc)
    assert_parity(res)
    assert res["energy"] > 0
    assert len(set(g["tri"][:, 0].tolist()) - {-1}) >= min(n_tri, 2)     # several triangles are seen


def test_axis_aligned_boxes_along_axes_offset_scene():
    """Axis-aligned boxes seen with an unrotated sensor on the LiDAR grid, so
    that the centre row and column of rays have exactly zero direction
    components (slab distances of +-1e30 on those axes), with scene and sensor
    moved far from the origin (the slab test's rounding bound grows with the
    origin's coordinates)."""
    torch, sonar = _gpu()
    off = np.array([256.0, -128.0, 64.0])
    parts = []
    for k, (cx, cy, z0, ex, ey, ez) in enumerate([(4.0, 0.3, -1.7, 0.5, 1.5, 1.2), (6.0, -1.1, -0.9, 1.0, 1.0, 1.6),
                                                   (8.5, 0.0, -2.5, 1.0, 4.0, 3.5), (5.0, 2.2, 0.4, 0.6, 0.8, 0.9),
                                                   (11.0, -3.0, -4.0, 2.0, 6.5, 7.0)]):
        v, t = S._box(cx + off[0], cy + off[1], z0 + off[2], ex, ey, ez)
        parts.append(M.mesh_from(v[t], rho=0.3 + 0.1 * k, phi=0.2 * k))
    mesh = M.concat(*parts)
    mesh.name = "aabb_offset"
    cfg = S.SensorConfig(n_h=16, n_v=8, rays_per_beam=1, grid_mode=1, jitter=0, n_range=512,
                         hfov=math.radians(60.0), vfov=math.radians(30.0))
    pose = S.pose(tuple(off))
    assert pose.rot == (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0)
    res, g, _ = run_parity(mesh, cfg, pose)
    assert_parity(res)
    centre = 4 * 17 + 8                      # el = 0, az = 0: direction (1, 0, 0) exactly
    assert g["tri"][centre, 0] >= 0
