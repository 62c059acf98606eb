"""Pins of the oracle's piecewise-linear sound-speed profile (a general
depth-dependent c(z); Sec. II-A: rays bend by Snell's law in a sound-speed
field): knots on one line reproduce the single-gradient model, equal speeds
reproduce straight rays, and single-bounce returns agree with a numerical
integration of the ray equations layer by layer (CPU only)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_2606_06130_amd import scenes as S
from tests import meshes as M


def _boxes_cfg(**kw):
    base = dict(n_h=16, n_v=8, rays_per_beam=4, n_range=512)
    base.update(kw)
    return S.sensor_seabed_boxes().replace(**base)


def _compare(a, b, amp_rel=1e-9):
    ok = (a["flags"] == 0) & (b["flags"] == 0)
    assert ok.mean() > 0.95
    for key in ("tri", "bin", "vis"):
        assert np.array_equal(a[key][ok], b[key][ok]), key
    da = np.abs(a["amp"][ok] - b["amp"][ok])
    assert np.all(da <= amp_rel * np.abs(b["amp"][ok]) + 1e-300)


def test_knots_on_one_line_equal_the_linear_profile():
    mesh = S.scene_seabed_boxes()
    sc = oracle.Scene(mesh)
    pose = S.pose_seabed_boxes()
    g, c0 = 0.05, 1500.0
    lin = _boxes_cfg(c_grad=g, c0=c0)
    z = [-9.0, -6.5, -3.25, -1.0, 0.5, 4.0]
    lay = _boxes_cfg(ssp=tuple((zz, c0 + g * zz) for zz in z))
    beams = np.arange(lin.n_beams)
    a = oracle.trace_beams(sc, lay, pose, beams)
    b = oracle.trace_beams(sc, lin, pose, beams)
    _compare(a, b)


def test_equal_speeds_equal_straight_rays():
    mesh = S.scene_seabed_boxes()
    sc = oracle.Scene(mesh)
    pose = S.pose_seabed_boxes()
    lay = _boxes_cfg(ssp=((-8.0, 1500.0), (-4.0, 1500.0), (-1.0, 1500.0)))
    beams = np.arange(lay.n_beams)
    _compare(oracle.trace_beams(sc, lay, pose, beams), oracle.trace_beams(sc, _boxes_cfg(), pose, beams), 1e-10)


def _ode_return(knots, z0, theta0, z_floor):
    """March the ray equations in the vertical plane through the layers:
    dx/ds = cos th, dz/ds = sin th, dth/ds = -c'(z) cos th / c(z),
    dT/ds = 1 / c(z), until the floor z = z_floor. Returns (x, T, s, th)."""
    kz = np.array([k[0] for k in knots])
    kc = np.array([k[1] for k in knots])

    def layer(z):
        i = int(np.searchsorted(kz, z, side="right")) - 1
        return min(max(i, 0), len(kz) - 2)

    def rhs_for(i):
        g = (kc[i + 1] - kc[i]) / (kz[i + 1] - kz[i])
        c0 = kc[i] - g * kz[i]

        def f(s, y):
            x, z, th, T = y
            c = c0 + g * z
            return [math.cos(th), math.sin(th), -g * math.cos(th) / c, 1.0 / c]
        return f

    y = np.array([0.0, z0, theta0, 0.0])
    s0 = 0.0
    i = layer(z0)
    if i > 0 and z0 == kz[i] and theta0 < 0:       # on a knot looking down: the layer below
        i -= 1
    for _ in range(64):
        if s0 > 400.0:
            return None, math.inf, s0, None
        lo = kz[i] if i > 0 else -np.inf
        hi = kz[i + 1] if i + 1 < len(kz) - 1 else np.inf

        def ev_floor(s, yy):
            return yy[1] - z_floor
        ev_floor.terminal = True

        def ev_lo(s, yy):
            return yy[1] - lo if np.isfinite(lo) else 1.0
        ev_lo.terminal = True
        ev_lo.direction = -1

        def ev_hi(s, yy):
            return yy[1] - hi if np.isfinite(hi) else -1.0
        ev_hi.terminal = True
        ev_hi.direction = 1
        r = solve_ivp(rhs_for(i), (s0, s0 + 100.0), y, events=(ev_floor, ev_lo, ev_hi), rtol=1e-12, atol=1e-13,
                      max_step=0.05)
        y, s0 = r.y[:, -1], r.t[-1]
        if len(r.t_events[0]):
            return y[0], y[3], s0, y[2]
        if len(r.t_events[1]):
            i -= 1
        elif len(r.t_events[2]):
            i += 1
    raise AssertionError("ray did not reach the floor")


@pytest.mark.parametrize("theta_deg", [-8.0, -20.0, -45.0, 3.0])
def test_single_bounce_matches_integrated_ray(theta_deg):
    """A flat floor at z = -12 under a three-layer profile (faster water above
    a slow channel); a ray at grazing angle theta in the x-z plane. The
    oracle's bin and phase carry its travel time, its amplitude the path
    length and the incidence angle: all agree with the integrated ray."""
    knots = ((-6.0, 1485.0), (-3.0, 1492.0), (0.0, 1502.0), (2.0, 1503.0))
    z_floor = -12.0
    floor = M.mesh_from([M.big_triangle_z(z_floor, half=400.0)], rho=0.5, phi=0.0)
    sc = oracle.Scene(floor)
    cfg = S.SensorConfig(n_h=8, n_v=8, rays_per_beam=1, n_range=4096, r_min=0.0, r_max=40.0, abs_db_per_m=0.0,
                         ssp=knots)
    pose = S.pose((0.0, 0.0, 0.0))
    th = math.radians(theta_deg)
    d0 = np.array([math.cos(th), 0.0, math.sin(th)])
    r = oracle.trace_one(sc, cfg, pose, np.zeros(3), d0)
    x, T, s, th_hit = _ode_return(knots, 0.0, th, z_floor)
    if T * 1502.0 > cfg.r_max:           # beyond the range window: no return
        assert r["bin"][0] == -1
        return
    assert r["flags"] == 0 and r["tri"][0] == 0
    c_ref = 1502.0
    dr = cfg.r_max / cfg.n_range
    assert r["bin"][0] == math.floor(c_ref * T / dr)
    # amplitude: sqrt(rho) |cos i| / (L^2 N_r), phase 2 pi f0 (2 T)
    want = math.sqrt(0.5) * abs(math.sin(th_hit)) / s ** 2 * np.exp(1j * 2 * math.pi * cfg.freq_hz * 2 * T)
    assert abs(r["amp"][0] - want) <= 1e-6 * abs(want)


def test_layered_profile_rejects_several_bounces_and_bad_knots():
    sc = oracle.Scene(M.mesh_from([M.big_triangle_z(-5.0)]))
    pose = S.pose((0.0, 0.0, 0.0))
    for cfg in (_boxes_cfg(ssp=((-5.0, 1490.0), (0.0, 1500.0)), max_bounces=2),
                _boxes_cfg(ssp=((0.0, 1490.0), (-5.0, 1500.0))),
                _boxes_cfg(ssp=((-5.0, 1490.0), (0.0, -1.0)))):
        with pytest.raises(ValueError):
            oracle.trace_beams(sc, cfg, pose, np.arange(4))
