"""Pins of the oracle's transmit-receive beam pattern and receive binning
(Sec. II-B: the contribution depends on the transmit-receive beam pattern)
against closed forms: pattern weights at the stratum centres, the mirror
geometry of a surface-wall path, and invariants between runs (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from paper_2606_06130_amd import scenes as S
from tests import meshes as M

LEVEL = S.pose((0.0, 0.0, 0.0))
LN2 = math.log(2.0)


def _cfg(**kw):
    base = dict(hfov=math.radians(40), vfov=math.radians(20), n_h=8, n_v=6, rays_per_beam=4, jitter=0,
                r_min=0.3, r_max=15.0, n_range=1024, max_bounces=1, k_d=1.0, k_s=0.0, c_grad=0.0)
    base.update(kw)
    return S.SensorConfig(**base)


def _lobe(da, de, dh, dv):
    return math.exp(-2.0 * LN2 * ((da / dh) ** 2 + (de / dv) ** 2))


@pytest.mark.parametrize("n_r", [1, 4, 16])
def test_pattern_weight_at_stratum_centres(n_r):
    """Single bounce: transmit and receive patterns both see the launch
    offset, so the weight is lobe^2 = exp(-4 ln2 ((a/dh)^2 + (e/dv)^2))."""
    sc = oracle.Scene(M.mesh_from([M.big_triangle_x(5.0)], rho=0.5, phi=0.3))
    cfg = _cfg(rays_per_beam=n_r)
    beams = np.arange(cfg.n_beams)
    plain = oracle.trace_beams(sc, cfg, LEVEL, beams)
    pat = oracle.trace_beams(sc, cfg.replace(flags=oracle.BEAM_PATTERN), LEVEL, beams)
    na, ne = {1: (1, 1), 4: (2, 2), 16: (4, 4)}[n_r]
    dh, dv = cfg.hfov / cfg.n_h, cfg.vfov / cfg.n_v
    ok = (plain["flags"] == 0) & (plain["bin"][:, 0] >= 0)
    assert ok.sum() > 0.9 * len(ok)
    for ri in np.nonzero(ok)[0]:
        j = ri % n_r
        a = ((j % na) + 0.5) / na * dh - 0.5 * dh
        e = ((j // na) + 0.5) / ne * dv - 0.5 * dv
        w = _lobe(a, e, dh, dv) ** 2
        assert abs(pat["amp"][ri, 0] - w * plain["amp"][ri, 0]) <= 1e-12 * abs(plain["amp"][ri, 0])
    if n_r == 4:                                   # offsets +-dh/4, +-dv/4: weight 2^-1/2 exactly
        r = np.abs(pat["amp"][ok, 0]) / np.abs(plain["amp"][ok, 0])
        assert np.allclose(r, 2 ** -0.5, rtol=1e-12)
    if n_r == 1:
        assert np.array_equal(pat["amp"], plain["amp"])


def _surface_wall():
    surf = M.mesh_from([M.big_triangle_z(2.0)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    wall = M.mesh_from([M.big_triangle_x(8.0)], rho=0.49, phi=0.7)
    return oracle.Scene(M.concat(surf, wall))


def _arrival_cell(cfg, d):
    """Closed-form second vertex of surface (z = 2) then wall (x = 8) and its
    direction from the sensor at the origin: (h, v, az offset, el offset)."""
    X1 = d * (2.0 / d[2])
    r = np.array([d[0], d[1], -d[2]])
    X2 = X1 + r * ((8.0 - X1[0]) / r[0])
    az = math.atan2(X2[1], X2[0])
    el = math.atan2(X2[2], math.hypot(X2[0], X2[1]))
    dh, dv = cfg.hfov / cfg.n_h, cfg.vfov / cfg.n_v
    h = int(math.floor((az + 0.5 * cfg.hfov) / dh))
    v = int(math.floor((el + 0.5 * cfg.vfov) / dv))
    return h, v, az - (-0.5 * cfg.hfov + (h + 0.5) * dh), el - (-0.5 * cfg.vfov + (v + 0.5) * dv)


def test_receive_beam_of_surface_wall_paths():
    """Rays up to the pressure-release surface, mirrored onto the wall: the
    second return arrives from the wall point, and receive binning puts it in
    the cell holding that direction (with both pattern weights applied)."""
    sc = _surface_wall()
    cfg = _cfg(hfov=math.radians(90), vfov=math.radians(40), n_h=16, n_v=8, rays_per_beam=4, jitter=1,
               max_bounces=2, k_d=0.7, k_s=0.3)
    beams = np.arange(cfg.n_beams)
    plain = oracle.trace_beams(sc, cfg, LEVEL, beams)
    rx = oracle.trace_beams(sc, cfg.replace(flags=oracle.RX_BEAMS), LEVEL, beams)
    both = oracle.trace_beams(sc, cfg.replace(flags=oracle.RX_BEAMS | oracle.BEAM_PATTERN), LEVEL, beams)
    dh, dv = cfg.hfov / cfg.n_h, cfg.vfov / cfg.n_v
    n_checked = moved = 0
    for ri in range(len(plain["flags"])):
        if plain["flags"][ri] or rx["flags"][ri] or list(plain["tri"][ri]) != [0, 1] or plain["bin"][ri, 1] < 0:
            continue
        b, j = divmod(ri, cfg.rays_per_beam)
        _, d = oracle.ray(cfg, LEVEL, b, j)
        h, v, da, de = _arrival_cell(cfg, d)
        assert rx["rxb"][ri, 1] == v * cfg.n_h + h
        assert rx["rxb"][ri, 0] == b                           # the first return stays in its launch beam
        # launch offsets from the ray's own angles
        az0 = math.atan2(d[1], d[0])
        el0 = math.atan2(d[2], math.hypot(d[0], d[1]))
        a0 = az0 - (-0.5 * cfg.hfov + (b % cfg.n_h + 0.5) * dh)
        e0 = el0 - (-0.5 * cfg.vfov + (b // cfg.n_h + 0.5) * dv)
        w = _lobe(a0, e0, dh, dv) * _lobe(da, de, dh, dv)
        assert abs(both["amp"][ri, 1] - w * plain["amp"][ri, 1]) <= 1e-10 * abs(plain["amp"][ri, 1])
        n_checked += 1
        moved += rx["rxb"][ri, 1] != b
    assert n_checked > 50 and moved > 10


@pytest.mark.parametrize("K", [2, 3])
def test_receive_binning_only_moves_contributions(K):
    """Receive binning changes where contributions land, nothing else: the
    per-ray records agree, bounce-1 returns keep their launch beam, the sum
    over all beams is unchanged, and every column is the sum of the
    contributions binned to it."""
    mesh = S.scene_seabed_boxes()
    sc = oracle.Scene(mesh)
    cfg = S.sensor_seabed_boxes().replace(n_h=16, n_v=8, rays_per_beam=4, n_range=256, max_bounces=K,
                                          k_d=0.7, k_s=0.3)
    pose = S.pose_seabed_boxes()
    beams = np.arange(cfg.n_beams)
    a = oracle.trace_beams(sc, cfg, pose, beams)
    b = oracle.trace_beams(sc, cfg.replace(flags=oracle.RX_BEAMS), pose, beams)
    for key in ("tri", "bin", "vis", "amp", "flags"):
        assert np.array_equal(a[key], b[key]), key
    launch = np.repeat(beams, cfg.rays_per_beam)
    assert np.array_equal(b["rxb"][:, 0], launch)
    assert np.array_equal(a["rxb"], np.repeat(launch[:, None], K, axis=1))
    assert abs(a["col_all"].sum() - b["col_all"].sum()) <= 1e-12 * np.abs(a["col_all"]).sum()
    vol = np.zeros_like(b["col_all"])
    for ri in range(len(launch)):
        for k in range(K):
            if b["bin"][ri, k] >= 0:
                vol[b["rxb"][ri, k], b["bin"][ri, k]] += b["amp"][ri, k]
    assert np.allclose(vol, b["col_all"], rtol=0, atol=1e-15 * np.abs(vol).max())
    moved = (b["rxb"][:, 1:] != launch[:, None]) & (b["bin"][:, 1:] >= 0)
    assert moved.sum() > 0


def test_beam_options_need_cell_beams_and_subsets_give_records_only():
    sc = _surface_wall()
    cfg = _cfg(max_bounces=2, k_s=0.3)
    # receive binning over a subset of beams: the records (the same as in a
    # run over every beam), no columns
    full = oracle.trace_beams(sc, cfg.replace(flags=oracle.RX_BEAMS), LEVEL, np.arange(cfg.n_beams))
    sub = oracle.trace_beams(sc, cfg.replace(flags=oracle.RX_BEAMS), LEVEL, np.arange(5, 9))
    rays = slice(5 * cfg.rays_per_beam, 9 * cfg.rays_per_beam)
    for key in ("tri", "bin", "vis", "rxb", "amp", "flags"):
        assert np.array_equal(sub[key], full[key][rays]), key
    assert not sub["col"].any()
    with pytest.raises(ValueError):
        oracle.trace_beams(sc, cfg.replace(flags=oracle.BEAM_PATTERN, grid_mode=1), LEVEL, np.arange(4))
