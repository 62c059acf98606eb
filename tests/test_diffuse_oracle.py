"""Pins of the oracle's Monte-Carlo continuation (Sec. II-B: stochastic
scattering and reverberation): the drawn directions follow the cosine lobe
and the Phong lobe (checked against their closed-form distributions), the
lobe choice follows k_s / (k_d + k_s), the draws are fixed by their counters,
and a very narrow Phong lobe reproduces the mirror paths (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2606_06130_amd import scenes as S
from tests import meshes as M


def _cfg(**kw):
    base = dict(n_h=16, n_v=8, rays_per_beam=4, n_range=512, max_bounces=3, k_d=0.7, k_s=0.3, phong_n=20.0,
                seed=77, flags=oracle.DIFFUSE_BOUNCE)
    base.update(kw)
    return S.sensor_seabed_boxes().replace(**base)


def _draws(cfg, n, kd, ks, rh, np_, k=1, ping=0):
    d = np.zeros((n, 3))
    c = np.zeros(n)
    lit = np.zeros(n, bool)
    for i in range(n):
        d[i], c[i], lit[i] = oracle.draw_continuation(cfg, ping, i, k, rh, np_, kd, ks)
    return d, c, lit


def _basis_azimuth(axis, d):
    """Azimuth of d around axis in an independent basis (Gram-Schmidt from x or y)."""
    a = np.asarray(axis, float)
    e = np.array([1.0, 0.0, 0.0]) if abs(a[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    u = e - a * (e @ a)
    u /= np.linalg.norm(u)
    v = np.cross(a, u)
    return np.arctan2(d @ v, d @ u)


@pytest.mark.parametrize("normal", [(0.0, 0.0, 1.0), (0.3, -0.5, -0.812403840463596), (0.0, 0.0, -1.0)])
def test_cosine_lobe(normal):
    cfg = _cfg()
    n = np.asarray(normal) / np.linalg.norm(normal)
    d, c, lit = _draws(cfg, 4000, 1.0, 0.0, (1.0, 0.0, 0.0), n)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)
    assert lit.all() and np.allclose(c, d @ n, atol=1e-14)
    assert stats.kstest(c ** 2, "uniform").pvalue > 1e-3                 # cos^2 a uniform: cosine-weighted
    az = _basis_azimuth(n, d)
    assert stats.kstest((az + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3


@pytest.mark.parametrize("n_exp", [1.0, 20.0, 200.0])
def test_phong_lobe(n_exp):
    cfg = _cfg(phong_n=n_exp)
    rh = np.array([0.6, 0.0, 0.8])
    d, c, lit = _draws(cfg, 4000, 0.0, 1.0, rh, (0.0, 0.0, 1.0))
    ca = d @ rh
    assert stats.kstest(ca ** (n_exp + 1.0), "uniform").pvalue > 1e-3   # (cos a)^(n+1) uniform
    assert np.array_equal(lit, c > 0)
    if n_exp >= 20:
        assert lit.mean() > 0.95


def test_lobe_choice_probability():
    cfg = _cfg(phong_n=5000.0)
    rh = np.array([0.6, 0.0, 0.8])
    d, _, _ = _draws(cfg, 6000, 0.7, 0.3, rh, (0.0, 0.0, 1.0))
    spec = (d @ rh) > 0.99                                                # the narrow Phong lobe
    assert stats.binomtest(int(spec.sum()), len(spec), 0.3).pvalue > 1e-3


def test_draws_fixed_by_their_counters():
    cfg = _cfg()
    a = oracle.draw_continuation(cfg, 3, 1234, 1, (0.0, 0.6, 0.8), (0.0, 0.0, 1.0), 0.5, 0.5)
    b = oracle.draw_continuation(cfg, 3, 1234, 1, (0.0, 0.6, 0.8), (0.0, 0.0, 1.0), 0.5, 0.5)
    assert np.array_equal(a[0], b[0])
    for other in (dict(ping=4), dict(ray=1235), dict(k=2)):
        args = dict(ping=3, ray=1234, k=1)
        args.update(other)
        c = oracle.draw_continuation(cfg, args["ping"], args["ray"], args["k"], (0.0, 0.6, 0.8), (0.0, 0.0, 1.0),
                                     0.5, 0.5)
        assert not np.array_equal(a[0], c[0])


def test_narrow_phong_lobe_reproduces_mirror_paths():
    """k_d = 0 and a very narrow lobe: the drawn continuation stays within
    ~1e-4 rad of the mirror, so paths hit the same facets and the returns
    agree closely; the amplitude weight sqrt(rho (k_d + k_s)) equals the
    mirror's sqrt(rho k_s)."""
    mesh = S.scene_seabed_boxes()
    sc = oracle.Scene(mesh)
    pose = S.pose_seabed_boxes()
    mc = _cfg(k_d=0.0, k_s=1.0, phong_n=1e9, max_bounces=2)
    mirror = mc.replace(flags=0)
    beams = np.arange(mc.n_beams)
    a = oracle.trace_beams(sc, mc, pose, beams)
    b = oracle.trace_beams(sc, mirror, pose, beams)
    ok = (a["flags"] == 0) & (b["flags"] == 0)
    assert ok.mean() > 0.9
    same = np.all(a["tri"][ok] == b["tri"][ok], axis=1)
    assert same.mean() > 0.99
    both = ok.copy()
    both[ok] = same
    m = (a["bin"][both] >= 0) & (b["bin"][both] >= 0)
    assert np.allclose(np.abs(a["amp"][both][m]), np.abs(b["amp"][both][m]), rtol=1e-3)


def test_monte_carlo_paths_differ_from_mirror_paths_and_keep_first_returns():
    surface = M.mesh_from([M.big_triangle_z(1.0)], rho=1.0, phi=0.0, mat=S.MAT_PRESSURE_RELEASE)
    mesh = M.concat(S.scene_seabed_boxes(), surface)
    sc = oracle.Scene(mesh)
    pose = S.pose_seabed_boxes()
    mc = _cfg()
    a = oracle.trace_beams(sc, mc, pose, np.arange(mc.n_beams))
    b = oracle.trace_beams(sc, mc.replace(flags=0), pose, np.arange(mc.n_beams))
    assert np.array_equal(a["tri"][:, 0], b["tri"][:, 0])               # the first hit is not drawn
    assert np.allclose(a["amp"][:, 0], b["amp"][:, 0], rtol=0, atol=0)
    has = (a["tri"][:, 1] >= 0) | (b["tri"][:, 1] >= 0)
    assert has.sum() > 30 and (a["tri"][has, 1] != b["tri"][has, 1]).mean() > 0.2
