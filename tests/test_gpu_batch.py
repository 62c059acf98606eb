"""Batched pings: one persistent launch over (ping, tile) items, hipGraph
replay and the launch-knob autotuner (needs an MI355X)."""
import math
import os
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


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mixed_items(base, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    items = []
    for i in range(n):
        nh, nv = ((8, 4), (16, 8), (33, 7), (64, 32))[int(rng.integers(0, 4))]
        nr = (1, 4, 8, 16)[int(rng.integers(0, 4))]
        cfg = base.replace(n_h=nh, n_v=nv, rays_per_beam=nr)
        yaw, pitch = rng.normal(0, 0.05), math.radians(55) + rng.normal(0, 0.05)
        pos = (rng.normal(0, 0.3), rng.normal(0, 0.3), rng.normal(0, 0.2))
        items.append((cfg, S.pose(pos, yaw, pitch, 0.0, ping=i)))
    return items


@pytest.mark.parametrize("physics", ["single", "multipath_gradient"])
def test_batch_equals_individual_pings(physics):
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    base = S.sensor_seabed_boxes()
    if physics == "multipath_gradient":
        base = base.replace(max_bounces=3, k_d=0.7, k_s=0.3, c_grad=0.05, n_range=512)
    sc = sonar.Scene(mesh)
    items = _mixed_items(base, 23, 7)
    batch = sonar.Batch(sc, items)
    batch.run(batch.options(blocks_per_cu=2, tiles_per_item=2))
    torch.cuda.synchronize()
    assert sc.status() == 0
    nz = 0
    for i, (cfg, pose) in enumerate(items):
        ref = sonar.ping(sc, cfg, pose)["volume"]
        torch.cuda.synchronize()
        a, b = batch.volumes[i].view(torch.float32), ref.view(torch.float32)
        assert torch.equal(a, b), (i, cfg.n_h, cfg.n_v, cfg.rays_per_beam)
        nz += int(torch.count_nonzero(b))
    assert nz > 0
    start, finish = batch.stamps()
    assert (finish > start).all()
    assert (start != np.uint64(2**64 - 1)).all()


def test_batch_graph_replay_matches_direct_launch():
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    base = S.sensor_seabed_boxes().replace(max_bounces=2, k_d=0.7, k_s=0.3, c_grad=0.05)
    sc = sonar.Scene(mesh)
    items = _mixed_items(base, 12, 11)
    batch = sonar.Batch(sc, items)
    batch.run()
    torch.cuda.synchronize()
    want = [v.clone() for v in batch.volumes]
    g = batch.graph(batch.options(blocks_per_cu=1, tiles_per_item=1))
    for rep in range(3):
        for v in batch.volumes:
            v.fill_(complex(float("nan"), 0.0))       # eager work between replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for i, v in enumerate(batch.volumes):
            assert torch.equal(v.view(torch.float32), want[i].view(torch.float32)), (rep, i)
    # descriptors updated in place: a replay picks up new poses
    items2 = [(cfg, S.Pose(tuple(np.asarray(p.position) + [0.0, 0.0, -0.5]), p.rot, p.ping)) for cfg, p in items]
    other = sonar.Batch(sc, items2)
    batch.desc.copy_(other.desc)
    # the copied descriptors point at `other`'s volumes
    g.launch()
    torch.cuda.synchronize()
    for i, (cfg, pose) in enumerate(items2):
        ref = sonar.ping(sc, cfg, pose)["volume"]
        torch.cuda.synchronize()
        assert torch.equal(other.volumes[i].view(torch.float32), ref.view(torch.float32))
    g.close()


def test_autotune_choice_keeps_results(tmp_path):
    """Every launch knob (workgroups of 1, 2, 4 waves; workgroups per CU;
    units per pop) gives the same volumes bit for bit; the autotuner's
    choice is one of them, cached with every candidate's time."""
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    sc = sonar.Scene(mesh)
    base = S.sensor_seabed_boxes().replace(max_bounces=2, k_d=0.7, k_s=0.3, c_grad=0.05)
    items = _mixed_items(base, 16, 3)
    batch = sonar.Batch(sc, items)
    batch.run()
    torch.cuda.synchronize()
    want = [v.clone() for v in batch.volumes]
    for wpb in (1, 2, 4):
        for bpc, tpi in ((1, 1), (3, 2), (6, 4)):
            for v in batch.volumes:
                v.fill_(complex(float("nan"), 0.0))
            batch.run(batch.options(blocks_per_cu=bpc, tiles_per_item=tpi, waves_per_block=wpb))
            torch.cuda.synchronize()
            for v, w in zip(batch.volumes, want):
                assert torch.equal(v.view(torch.float32), w.view(torch.float32)), (wpb, bpc, tpi)
            start, finish = batch.stamps()
            assert (finish > start).all()
    os.environ["SONAR_AUTOTUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        best, ms = batch.autotune()
        assert best.blocks_per_cu >= 1 and best.tiles_per_item in (1, 2, 4) and ms > 0
        assert best.waves_per_block in (1, 2, 4)
        best2, ms2 = batch.autotune()          # cached
        assert (best2.blocks_per_cu, best2.tiles_per_item, best2.waves_per_block, ms2) == \
            (best.blocks_per_cu, best.tiles_per_item, best.waves_per_block, pytest.approx(ms, rel=1e-5))
        lines = (tmp_path / "tune.txt").read_text().strip().splitlines()
        cands = [l for l in lines if l.startswith("cand:")]
        assert {int(l.split()[3]) for l in cands} == {1, 2, 4}
        assert len(cands) >= 9
    finally:
        del os.environ["SONAR_AUTOTUNE_CACHE"]
    batch.run(best)
    torch.cuda.synchronize()
    for v, w in zip(batch.volumes, want):
        assert torch.equal(v.view(torch.float32), w.view(torch.float32))
    _log("autotuned", best.blocks_per_cu, best.tiles_per_item, best.waves_per_block, ms)


def test_batch_rejects_mixed_physics():
    torch, sonar = _gpu()
    sc = sonar.Scene(S.scene_seabed_boxes())
    items = [(S.sensor_seabed_boxes(), S.pose_seabed_boxes()),
             (S.sensor_seabed_boxes().replace(max_bounces=2), S.pose_seabed_boxes())]
    with pytest.raises(sonar.SonarError) as e:
        sonar.Batch(sc, items)
    assert e.value.status == sonar.SONAR_E_INVALID


@pytest.mark.parametrize("physics", ["single", "multipath_gradient"])
def test_batch_detection_equals_individual_ping_detect(physics):
    """Batched pings with the fused CFAR test and one batched emission give,
    per ping, the volume and the point cloud of sonar_ping_detect on its own;
    graph replays repeat them with eager work in between."""
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    base = S.sensor_seabed_boxes()
    if physics == "multipath_gradient":
        base = base.replace(max_bounces=2, k_d=0.7, k_s=0.3, c_grad=0.05, n_range=512)
    sc = sonar.Scene(mesh)
    items = _mixed_items(base, 17, 5)
    M = 3
    batch = sonar.Batch(sc, items)
    batch.detect(train=8, guard=2, max_per_beam=M)
    want = []
    for cfg, pose in items:
        det = sonar.Detector(cfg, train=8, guard=2, max_per_beam=M)
        vol = sonar.alloc_outputs(cfg)["volume"]
        det.ping_detect(sc, vol, pose)
        pts, cnt = det.fetch()
        want.append((vol.clone(), pts.copy(), cnt))
    total = sum(w[2] for w in want)
    assert total > 0
    _log(physics, "points per ping", [w[2] for w in want])

    def check(tag):
        for i, (vol, pts, cnt) in enumerate(want):
            assert torch.equal(batch.volumes[i].view(torch.float32), vol.view(torch.float32)), (tag, i)
            got, c = batch.point_cloud(i)
            assert c == cnt, (tag, i, c, cnt)
            assert np.array_equal(got, pts), (tag, i)

    batch.run(batch.options(blocks_per_cu=2, tiles_per_item=2))
    torch.cuda.synchronize()
    assert sc.status() == 0
    check("direct")
    g = batch.graph()
    for rep in range(3):
        for v in batch.volumes:
            v.fill_(complex(float("nan"), 0.0))
        for p in batch.points:
            p.fill_(-7)
        batch.counts.fill_(-1)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        check(f"replay {rep}")
    g.close()


def test_batch_detection_rejects_mismatched_parameters():
    torch, sonar = _gpu()
    sc = sonar.Scene(S.scene_seabed_boxes())
    items = _mixed_items(S.sensor_seabed_boxes(), 4, 2)
    batch = sonar.Batch(sc, items)
    batch._P[1].n_h += 1          # no longer the layout the descriptors were prepared for
    with pytest.raises(sonar.SonarError) as e:
        batch.detect()
    assert e.value.status == sonar.SONAR_E_INVALID


def test_batch_matches_oracle_multipath_harbor():
    """Ten pings of the lawnmower trajectory over the 1,991,680-triangle
    multipath scene (3 bounces, c(z) = 1500 + 0.05 z) in one persistent launch
    with the fused CA-CFAR: mixed layouts (64 x 32 to 256 x 128 beams), 4-16
    rays per beam and mixed bin counts (512, 777, 1,024). Each ping carries the
    oracle's flagged rays as its mask and records its rays; 256 sampled beams
    per ping are compared with the oracle ray by ray (triangle, bin and
    visibility bit-exact, contributions) and column by column (volume,
    G-buffer, incoherent channels), and every ping's point cloud with the
    oracle's detection on the batch's own volume."""
    import oracle
    from tests.parity import compare_points, compare_rays, mask_words, ray_ids, rel_l2
    torch, sonar = _gpu()
    mesh = S.scene_harbor_multipath()
    traj = S.lawnmower_batch()
    pick = [0, 37, 70, 101, 128, 150, 190, 205, 231, 255]
    bins = (1024, 512, 777)
    items = [(traj[p][0].replace(n_range=bins[i % 3]), traj[p][1]) for i, p in enumerate(pick)]
    layouts = {(c.n_h, c.rays_per_beam) for c, _ in items}
    assert len({c.n_h for c, _ in items}) == 3 and len({c.rays_per_beam for c, _ in items}) == 3, layouts
    sc = sonar.Scene(mesh)
    osc = oracle.Scene(mesh)
    batch = sonar.Batch(sc, items)
    rng = np.random.Generator(np.random.PCG64(77))
    orcs, sampled = [], []
    for i, (cfg, pose) in enumerate(items):
        beams = np.sort(rng.choice(cfg.n_beams, 256, replace=False))
        orc = oracle.trace_beams(osc, cfg, pose, beams, want_incoh=True, want_gbuf=True)
        rays = ray_ids(beams, cfg.rays_per_beam)
        mask = torch.from_numpy(mask_words(cfg.n_rays, rays[orc["flags"] != 0])).cuda()
        batch.set_outputs(i, gbuffer=True, incoh=True, record=True, ray_mask=mask)
        orcs.append(orc)
        sampled.append((beams, rays))
    batch.detect()
    batch.run(batch.options(blocks_per_cu=2, tiles_per_item=1))
    torch.cuda.synchronize()
    assert sc.status() == 0
    flagged = total_rays = im_energy = 0
    for i, (cfg, pose) in enumerate(items):
        beams, rays = sampled[i]
        orc = orcs[i]
        ex = batch.extras[i]
        g = {k: v.cpu().numpy() for k, v in ex.items() if k != "ray_mask"}
        res = compare_rays(g, orc, rays)
        for key in ("tri_mismatch", "bin_mismatch", "vis_mismatch"):
            assert res[key] == 0, (i, res)
        ok = orc["flags"] == 0
        if np.abs(orc["amp"][ok]).sum() > 0:
            assert rel_l2(g["amp"][rays][ok], orc["amp"][ok]) <= 1e-4, i
        vol = batch.volumes[i].cpu().numpy().reshape(cfg.n_beams, cfg.n_range)
        assert rel_l2(vol[beams], orc["col"]) <= 1e-4, (i, res)
        inc = g["incoh"].reshape(2, cfg.n_beams, cfg.n_range)[:, beams]
        assert rel_l2(inc[0], orc["incoh"][:, 0]) <= 1e-4, i
        if orc["incoh"][:, 1].sum() > 0:
            assert rel_l2(inc[1], orc["incoh"][:, 1]) <= 1e-4, i
        im_energy += float(orc["incoh"][:, 1].sum())
        assert np.abs(g["gbuffer"].reshape(cfg.n_beams, 8)[beams] - orc["gbuf"]).max() <= 1e-5, i
        flagged += res["flagged"]
        total_rays += res["rays"]
        pts, n = batch.point_cloud(i)
        o = oracle.detect(vol, cfg, pose, np.arange(cfg.n_beams))
        compared = compare_points(pts, n, o, np.arange(cfg.n_beams))
        assert compared >= 0.99 * cfg.n_beams, (i, compared)
        _log("batch ping", i, cfg.n_h, cfg.n_v, cfg.rays_per_beam, cfg.n_range, "flagged", res["flagged"], "points", n)
    assert im_energy > 0
    assert flagged <= 0.01 * 5 * total_rays, (flagged, total_rays)
