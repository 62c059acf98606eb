"""Pins of the oracle's G-buffer and incoherent channels against closed forms
(CPU only).

The G-buffer (per beam, over its unflagged first-bounce hits in range: mean
range / r_max, mean cos incidence, mean reflectivity, mean facet normal facing
the ray, hit count / rays per beam, and the vertical component of the beam
axis) is the learned surrogate's whole input; the incoherent channels split
sum |A|^2 into first-bounce and later-bounce returns (Sec. II-B: scattering
from incidence angle and material, a bounded number of secondary
reflections). Every expected value below is written from the geometry alone:
ray directions from the stratum centres of the sensor grid, ranges and
incidence from plane distances, the normal from the plane's orientation.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2606_06130_amd import scenes as S
from tests import meshes as M

REL = 1e-12


def _cfg(**kw):
    base = dict(hfov=math.radians(30), vfov=math.radians(20), n_h=5, n_v=3, rays_per_beam=4, jitter=0,
                r_min=0.3, r_max=15.0, n_range=512, max_bounces=1, k_d=1.0, k_s=0.0, c_grad=0.0)
    base.update(kw)
    return S.SensorConfig(**base)


def _strata(n_r):
    return {1: (1, 1), 2: (2, 1), 4: (2, 2), 8: (4, 2), 16: (4, 4)}[n_r]


def _sensor_dirs(cfg, b):
    """Sensor-frame unit directions of beam b's rays at the stratum centres,
    and the beam-centre direction."""
    na, ne = _strata(cfg.rays_per_beam)
    h, v = b % cfg.n_h, b // cfg.n_h
    dh, dv = cfg.hfov / cfg.n_h, cfg.vfov / cfg.n_v
    out = []
    for j in range(cfg.rays_per_beam):
        ja, je = j % na, j // na
        az = -cfg.hfov / 2 + (h + (ja + 0.5) / na) * dh
        el = -cfg.vfov / 2 + (v + (je + 0.5) / ne) * dv
        out.append((math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)))
    azc = -cfg.hfov / 2 + (h + 0.5) * dh
    elc = -cfg.vfov / 2 + (v + 0.5) * dv
    return np.array(out), np.array([math.cos(elc) * math.cos(azc), math.cos(elc) * math.sin(azc), math.sin(elc)])


def _pitched(p):
    """Sensor->world rotation of a sensor pitched down by p (columns: sensor
    axes in the world frame), written out, and the matching pose."""
    cp, sp = math.cos(p), math.sin(p)
    R = np.array([[cp, 0.0, sp], [0.0, 1.0, 0.0], [-sp, 0.0, cp]])
    return R, S.Pose((0.0, 0.0, 0.0), tuple(R.reshape(-1)), 0)


def _close(a, b, rel=REL, atol=1e-15):
    return abs(a - b) <= rel * abs(b) + atol


@pytest.mark.parametrize("d", [3.0, 7.25])
@pytest.mark.parametrize("flip", [False, True])
def test_gbuffer_plane_perpendicular_to_boresight(d, flip):
    """Plane x = d, level sensor: range d / cos(psi), cos incidence cos(psi),
    the normal facing the ray (-1, 0, 0) whichever way the triangle is wound,
    every ray a hit, beam axis z = sin(el_centre); I1 = sum over the rays in
    a bin of (sqrt(rho) cos^3(psi) / (d^2 N_r) 10^(-0.3 * 2R / 20))^2, Im = 0."""
    rho = float(np.float32(0.64))
    tri = M.big_triangle_x(d)
    if flip:
        tri = [tri[0], tri[2], tri[1]]
    cfg = _cfg()
    sc = oracle.Scene(M.mesh_from([tri], rho=rho, phi=0.5))
    beams = np.arange(cfg.n_beams)
    r = oracle.trace_beams(sc, cfg, S.pose((0.0, 0.0, 0.0)), beams, want_gbuf=True, want_incoh=True)
    assert (r["flags"] == 0).all()
    dr = (cfg.r_max - cfg.r_min) / cfg.n_range
    for b in beams:
        dirs, axis = _sensor_dirs(cfg, b)
        cpsi = dirs[:, 0]
        R = d / cpsi
        g = r["gbuf"][b]
        assert _close(g[0], np.mean(R / cfg.r_max))
        assert _close(g[1], np.mean(cpsi))
        assert _close(g[2], rho)
        assert g[3] == -1.0 and g[4] == 0.0 and g[5] == 0.0
        assert g[6] == 1.0
        assert _close(g[7], axis[2])
        i1 = np.zeros(cfg.n_range)
        for Rj, cj in zip(R, cpsi):
            a = math.sqrt(rho) * cj ** 3 / (d * d * cfg.rays_per_beam) * 10 ** (-0.3 * 2 * Rj / 20)
            i1[math.floor((Rj - cfg.r_min) / dr)] += a * a
        np.testing.assert_allclose(r["incoh"][b, 0], i1, rtol=REL, atol=0)
        assert not r["incoh"][b, 1].any()


@pytest.mark.parametrize("flip", [False, True])
def test_gbuffer_pitched_over_seabed(flip):
    """Sensor pitched 35 deg down over a seabed plane z = -h: a ray with world
    direction w hits at range h / (-w_z) with cos incidence -w_z, the normal
    facing it is (0, 0, 1); rays beyond r_max add nothing, so the hit count is
    the number of rays with h / (-w_z) < r_max; the beam axis z is the world z
    of the beam-centre direction, -sin(p) cos(el) cos(az) + cos(p) sin(el)."""
    h, p = 5.0, math.radians(35.0)
    rho = float(np.float32(0.3))
    tri = M.big_triangle_z(-h)
    if flip:
        tri = [tri[0], tri[2], tri[1]]
    cfg = _cfg(hfov=math.radians(60), vfov=math.radians(40), n_h=6, n_v=4, r_max=11.0)
    R3, pose = _pitched(p)
    sc = oracle.Scene(M.mesh_from([tri], rho=rho, phi=0.1))
    beams = np.arange(cfg.n_beams)
    r = oracle.trace_beams(sc, cfg, pose, beams, want_gbuf=True, want_incoh=True)
    assert (r["flags"] == 0).all()
    partial = 0
    for b in beams:
        dirs, axis = _sensor_dirs(cfg, b)
        wz = dirs @ R3[2]
        down = wz < 0
        R = np.where(down, h / np.where(down, -wz, 1.0), np.inf)
        hit = (R >= cfg.r_min) & (R < cfg.r_max)
        g = r["gbuf"][b]
        n_hit = int(hit.sum())
        assert g[6] == n_hit / cfg.rays_per_beam
        partial += 0 < n_hit < cfg.rays_per_beam
        assert _close(g[7], -math.sin(p) * axis[0] + math.cos(p) * axis[2])
        if n_hit == 0:
            assert not g[:6].any()
            continue
        assert _close(g[0], np.mean(R[hit] / cfg.r_max))
        assert _close(g[1], np.mean(-wz[hit]))
        assert _close(g[2], rho)
        assert g[3] == 0.0 and g[4] == 0.0 and g[5] == 1.0
    assert partial > 0          # some beams straddle r_max: the count is not always 0 or N_r


def test_gbuffer_half_covered_beam_and_occluder():
    """The centre beam of an odd row (azimuths +-dth/4 at the stratum
    centres): a half-plane y >= 0 at x = d1 in front of a full plane at
    x = d2. Alone, the half-plane gives a hit fraction of 1/2 and means over
    the two rays that reach it; with the far plane behind it, every ray hits
    and the mean range mixes d1 / cos(psi) and d2 / cos(psi) two and two
    (nearest hit, so the far plane does not show through the near one)."""
    d1, d2 = 4.0, 9.0
    rho1, rho2 = float(np.float32(0.2)), float(np.float32(0.8))
    half = [[d1, 0.0, -60.0], [d1, 0.0, 60.0], [d1, 60.0, 0.0]]
    cfg = _cfg(n_h=3, n_v=1, hfov=math.radians(12), vfov=math.radians(6))
    b = 1
    dirs, _ = _sensor_dirs(cfg, b)
    left = dirs[:, 1] > 0                     # azimuth toward +y: the half-plane's side
    assert left.sum() == 2
    cpsi = dirs[:, 0]
    pose = S.pose((0.0, 0.0, 0.0))

    r = oracle.trace_beams(oracle.Scene(M.mesh_from([half], rho=rho1)), cfg, pose, np.array([b]), want_gbuf=True)
    assert (r["flags"] == 0).all()
    g = r["gbuf"][0]
    assert g[6] == 0.5
    assert _close(g[0], np.mean(d1 / cpsi[left] / cfg.r_max))
    assert _close(g[1], np.mean(cpsi[left]))
    assert _close(g[2], rho1)

    mesh = M.concat(M.mesh_from([half], rho=rho1), M.mesh_from([M.big_triangle_x(d2)], rho=rho2))
    r = oracle.trace_beams(oracle.Scene(mesh), cfg, pose, np.array([b]), want_gbuf=True)
    assert (r["flags"] == 0).all()
    g = r["gbuf"][0]
    R = np.where(left, d1, d2) / cpsi
    assert g[6] == 1.0
    assert _close(g[0], np.mean(R / cfg.r_max))
    assert _close(g[1], np.mean(cpsi))
    assert _close(g[2], np.mean(np.where(left, rho1, rho2)))
    assert list(r["tri"][:, 0]) == [1 if not l else 0 for l in left]


def test_incoherent_split_vertical_surface_seabed_path():
    """Sensor looking straight up between a pressure-release surface at
    z = +s and a rough seabed at z = -h (boresight emitter of the LiDAR
    grid), 3 bounces: surface (range s) -> seabed (its return would arrive
    from behind the sensor: outside the field of view, no contribution) ->
    surface (returns down the vertical, range 2s + h). Closed forms of the
    amplitudes (Sec. II-B weights: the surface's lobe 1 with sign -1, the
    seabed's sqrt(rho k_s) on the mirror chain, spreading 1 / (L_out L_back),
    absorption on the total path): the first lands in I1, the third in Im."""
    h, s = 3.0, 2.0
    rho, kd, ks, n = float(np.float32(0.6)), 0.7, 0.3, 20.0
    surf = M.mesh_from([M.big_triangle_z(s)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    bed = M.mesh_from([M.big_triangle_z(-h)], rho=rho, phi=0.0)
    cfg = S.SensorConfig(hfov=math.radians(2), vfov=math.radians(2), n_h=2, n_v=2, rays_per_beam=1, jitter=0,
                         grid_mode=1, r_min=0.3, r_max=15.0, n_range=1024, max_bounces=3, k_d=kd, k_s=ks,
                         phong_n=n)
    R = np.array([[0.0, 0.0, -1.0], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0]])     # boresight +z, exactly
    pose = S.Pose((0.0, 0.0, 0.0), tuple(R.reshape(-1)), 0)
    centre = 1 * 3 + 1                                                      # emitter on the boresight
    r = oracle.trace_beams(oracle.Scene(M.concat(surf, bed)), cfg, pose, np.array([centre]), want_incoh=True)
    assert r["flags"][0] == 0
    assert list(r["tri"][0]) == [0, 1, 0]
    assert list(r["vis"][0]) == [1, 0, 1]
    assert r["bin"][0, 1] == -1 and r["amp"][0, 1] == 0
    dr = (cfg.r_max - cfg.r_min) / cfg.n_range

    def att(L):
        return 10 ** (-0.3 * L / 20)
    a1 = -1.0 * att(2 * s) / (s * s)
    Lo3, Lb3 = s + (s + h) + (h + s), s
    a3 = (-1.0) * math.sqrt(rho * ks) * (-1.0) * att(Lo3 + Lb3) / (Lo3 * Lb3)
    bins = [math.floor((s - cfg.r_min) / dr), math.floor(((Lo3 + Lb3) / 2 - cfg.r_min) / dr)]
    assert [r["bin"][0, 0], r["bin"][0, 2]] == bins
    for k, a, L in ((0, a1, 2 * s), (2, a3, Lo3 + Lb3)):
        assert _close(abs(r["amp"][0, k]), abs(a))
        # the sign of the chain: arg(A) - 2 pi f0 T is 0 or pi
        ph = np.angle(r["amp"][0, k] * np.exp(-2j * math.pi * cfg.freq_hz * L / cfg.c0))
        assert abs(abs(ph) - (0.0 if a > 0 else math.pi)) < 1e-6
    inc = r["incoh"][0]
    want1 = np.zeros(cfg.n_range)
    want1[bins[0]] = a1 * a1
    wantm = np.zeros(cfg.n_range)
    wantm[bins[1]] = a3 * a3
    np.testing.assert_allclose(inc[0], want1, rtol=REL, atol=0)
    np.testing.assert_allclose(inc[1], wantm, rtol=REL, atol=0)
