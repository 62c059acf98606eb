"""Pins of the oracle's retro-chain returns (Sec. II-B: secondary reflections
beyond the direct return; a vertex after the first also scatters back along
its own outgoing chain reversed): closed forms for a vertical ray between a
seabed and a pressure-release surface and for an oblique ray into a
wall-seabed corner (geometry, spreading, both passes of the chain's weights,
the backscatter lobe, time and phase), and accumulation checks (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from paper_2606_06130_amd import scenes as S
from tests import meshes as M

RETRO = 8


def f32(x):
    """Facet materials are stored in FP32."""
    return float(np.float32(x))


def _cfg(**kw):
    base = dict(n_h=8, n_v=8, rays_per_beam=1, n_range=2048, r_min=0.0, r_max=40.0, abs_db_per_m=0.05,
                max_bounces=2, k_d=0.6, k_s=0.4, phong_n=8.0, flags=RETRO)
    base.update(kw)
    return S.SensorConfig(**base)


def test_vertical_ray_between_seabed_and_surface():
    """Straight down onto a seabed at -h, mirrored up to a pressure-release
    surface at +s: the second vertex's retro-chain return has path 2 (2h + s),
    the seabed's specular weight twice, the surface's -1, and backscatter
    exactly along the mirror (lobe 1)."""
    h, s = 6.0, 2.0
    rho_b = f32(0.45)
    seabed = M.mesh_from([M.big_triangle_z(-h)], rho=rho_b, phi=0.7)
    surface = M.mesh_from([M.big_triangle_z(s)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    sc = oracle.Scene(M.concat(seabed, surface))
    cfg = _cfg()
    r = oracle.trace_one(sc, cfg, S.pose((0.0, 0.0, 0.0)), np.zeros(3), (0.0, 0.0, -1.0))
    assert r["flags"] == 0 and list(r["tri"]) == [0, 1]
    assert r["rbin"][0] == -1                                   # the first vertex has no chain to retrace
    L = 2 * h + s
    c = cfg.c0
    dr = (cfg.r_max - cfg.r_min) / cfg.n_range
    assert r["rbin"][1] == math.floor((L - cfg.r_min) / dr)
    att = 10 ** (-cfg.abs_db_per_m * 2 * L / 20)
    mag = rho_b * cfg.k_s * 1.0 * att / L ** 2                 # W^2 = rho_b k_s; pressure release: rho k_s = 1
    want = -mag * np.exp(1j * 2 * math.pi * cfg.freq_hz * 2 * L / c)
    assert abs(r["ramp"][1] - want) <= 1e-9 * mag          # the phase argument is ~4e4 rad


@pytest.mark.parametrize("el_deg,n_exp", [(-20.0, 8.0), (-35.0, 1.0), (-8.0, 30.0)])
def test_oblique_ray_into_a_wall_seabed_corner(el_deg, n_exp):
    d_wall, h = 9.0, 8.0
    rho_w, rho_b, phi_b = f32(0.8), f32(0.35), f32(-1.1)
    wall = M.mesh_from([M.big_triangle_x(d_wall)], rho=rho_w, phi=0.3)
    seabed = M.mesh_from([M.big_triangle_z(-h)], rho=rho_b, phi=phi_b)
    sc = oracle.Scene(M.concat(wall, seabed))
    cfg = _cfg(phong_n=n_exp, r_max=60.0, n_range=4096)
    el = math.radians(el_deg)
    d0 = np.array([math.cos(el), 0.0, math.sin(el)])
    # the chain by hand: wall first, then the seabed along the mirror
    t1 = d_wall / d0[0]
    X1 = t1 * d0
    assert X1[2] > -h
    r1 = np.array([-d0[0], d0[1], d0[2]])
    t2 = (-h - X1[2]) / r1[2]
    L = t1 + t2
    cos_i = -r1[2]
    rh2 = np.array([r1[0], r1[1], -r1[2]])
    lobe = max(0.0, -float(rh2 @ r1))
    fsc = rho_b * (cfg.k_d * cos_i ** 2 + cfg.k_s * lobe ** n_exp)
    att = 10 ** (-cfg.abs_db_per_m * 2 * L / 20)
    mag = rho_w * cfg.k_s * math.sqrt(fsc) * att / L ** 2
    want = mag * np.exp(1j * (2 * math.pi * cfg.freq_hz * 2 * L / cfg.c0 + phi_b))
    r = oracle.trace_one(sc, cfg, S.pose((0.0, 0.0, 0.0)), np.zeros(3), d0)
    assert r["flags"] == 0 and list(r["tri"]) == [0, 1]
    dr = (cfg.r_max - cfg.r_min) / cfg.n_range
    assert r["rbin"][1] == math.floor(L / dr)
    assert abs(r["ramp"][1] - want) <= 1e-9 * mag


def _surface_wall():
    """A pressure-release surface over a rough wall, looked at slightly upward."""
    surf = M.mesh_from([M.big_triangle_z(2.0)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    wall = M.plane_grid_x(8.0, -6.0, 6.0, -8.0, 2.0, 40, np.random.Generator(np.random.PCG64(1)))
    cfg = S.SensorConfig(n_h=32, n_v=16, rays_per_beam=2, n_range=1024, max_bounces=3, k_d=0.7, k_s=0.3,
                         vfov=math.radians(60))
    return oracle.Scene(M.concat(surf, wall)), S.pose((0.0, 0.0, 0.0), pitch_down=math.radians(-10)), cfg


def test_retro_returns_add_to_the_columns_and_change_nothing_else():
    sc, pose, base = _surface_wall()
    beams = np.arange(base.n_beams)
    off = oracle.trace_beams(sc, base, pose, beams, want_incoh=True)
    on = oracle.trace_beams(sc, base.replace(flags=RETRO), pose, beams, want_incoh=True)
    assert (off["rbin"] == -1).all()
    for key in ("tri", "bin", "vis", "flags"):
        assert np.array_equal(on[key], off[key])
    assert np.array_equal(on["amp"], off["amp"])
    assert (on["rbin"][:, 0] == -1).all() and (on["rbin"][:, 1:] >= 0).sum() > 300
    # the columns gain exactly the retro contributions of unflagged rays
    ok = on["flags"] == 0
    nr, nb = base.rays_per_beam, base.n_range
    extra = np.zeros((base.n_beams, nb), complex)
    extra_i = np.zeros((base.n_beams, nb))
    for ray in np.flatnonzero(ok):
        for k in range(1, base.max_bounces):
            b = on["rbin"][ray, k]
            if b >= 0:
                extra[ray // nr, b] += on["ramp"][ray, k]
                extra_i[ray // nr, b] += abs(on["ramp"][ray, k]) ** 2
    assert np.allclose(on["col"] - off["col"], extra, rtol=0, atol=1e-15)
    assert np.allclose(on["incoh"][:, 1] - off["incoh"][:, 1], extra_i, rtol=0, atol=1e-20)
    assert np.array_equal(on["incoh"][:, 0], off["incoh"][:, 0])


def test_retro_returns_with_receive_binning_stay_in_the_launch_beam():
    sc, pose, base = _surface_wall()
    beams = np.arange(base.n_beams)
    rx = oracle.trace_beams(sc, base.replace(flags=2), pose, beams)
    both = oracle.trace_beams(sc, base.replace(flags=2 | RETRO), pose, beams)
    assert np.array_equal(both["ramp"], oracle.trace_beams(sc, base.replace(flags=RETRO), pose, beams)["ramp"])
    ok = both["flags"] == 0
    extra = np.zeros((base.n_beams, base.n_range), complex)
    for ray in np.flatnonzero(ok):
        for k in range(1, base.max_bounces):
            if both["rbin"][ray, k] >= 0:
                extra[ray // base.rays_per_beam, both["rbin"][ray, k]] += both["ramp"][ray, k]
    assert np.allclose(both["col"] - rx["col"], extra, rtol=0, atol=1e-15)
