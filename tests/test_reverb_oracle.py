"""Pins of the volume-reverberation-and-noise oracle (Sec. II-B: water-column
backscatter, speckle): its generator against the C oracle's SplitMix64
(pinned to published outputs), the Box-Muller samples' distribution, the
mean power law in range, determinism and counter independence (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import reverb as R
from paper_2606_06130_amd import scenes as S


def _cfg(**kw):
    base = dict(hfov=math.radians(60), vfov=math.radians(20), n_h=32, n_v=16, rays_per_beam=1, r_min=0.5,
                r_max=15.0, n_range=256, abs_db_per_m=0.3)
    base.update(kw)
    return S.SensorConfig(**base)


def test_vectorised_splitmix_equals_the_pinned_generator():
    seed = 0x1234ABCD
    ns = [1, 2, 3, 17, 1 << 20, (1 << 43) + 5, (1 << 63) + 11]
    got = R.splitmix64(seed, np.array(ns, np.uint64))
    assert [int(x) for x in got] == [oracle.splitmix64_nth(seed, n) for n in ns]


def test_counter_layout():
    c = R.counters(3, [0, 1, 5], [0, 7])
    assert int(c[0, 0]) == 3 << 43 and int(c[2, 1]) == (3 << 43) ^ (5 << 12) ^ 7


def test_box_muller_samples_are_standard_normal():
    g = R.gaussians(99, 0, np.arange(512), np.arange(256)).reshape(-1)
    for part in (g.real, g.imag):
        assert abs(part.mean()) < 4 / math.sqrt(part.size)
        assert abs(part.var() - 1.0) < 6 * math.sqrt(2.0 / part.size)
        assert stats.kstest(part, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(g.real, g.imag)[0, 1]) < 4 / math.sqrt(g.size)
    # |g|^2 / 2 is exponential with unit mean (Rayleigh amplitude: speckle)
    assert stats.kstest(np.abs(g) ** 2 / 2, "expon").pvalue > 1e-3


def test_mean_power_law_in_range():
    cfg = _cfg()
    bins = np.array([0, 50, 200])
    P = R.mean_power(cfg, [0], bins, -40.0, 0.0)[0]
    dr = (cfg.r_max - cfg.r_min) / cfg.n_range
    r = cfg.r_min + (bins + 0.5) * dr
    # two cells of one beam: (r2 / r1)^2 spreading and two-way absorption over the difference
    want = (r[1] / r[0]) ** 2 * 10 ** (-0.3 * 2 * (r[0] - r[1]) / 10)
    assert abs(P[0] / P[1] - want) < 1e-12 * want
    # one cell: s_v dth_h dth_v dr cos(el) / r^2 with absorption
    el = -0.5 * cfg.vfov + 0.5 * cfg.vfov / cfg.n_v
    one = 1e-4 * (cfg.hfov / cfg.n_h) * (cfg.vfov / cfg.n_v) * dr * math.cos(el) / r[2] ** 2 * 10 ** (-0.06 * r[2])
    assert abs(P[2] - one) < 1e-12 * one
    assert np.allclose(R.mean_power(cfg, [0, 5], bins, -300.0, 2.5e-9), 2.5e-9, rtol=1e-12)


def test_sample_power_matches_mean_power():
    cfg = _cfg(n_h=64, n_v=64)
    nb = cfg.n_beams
    out = R.add(np.zeros((nb, cfg.n_range)), cfg, 0, -30.0, 1e-12, 7)
    P = R.mean_power(cfg, np.arange(nb), np.arange(cfg.n_range), -30.0, 1e-12)
    ratio = (np.abs(out) ** 2 / P).reshape(nb, -1)
    m = ratio.mean(axis=0)                       # per bin, over 4,096 beams: exponential(1) means
    assert np.all(np.abs(m - 1.0) < 6 / math.sqrt(nb))


def test_deterministic_additive_and_counter_independent():
    cfg = _cfg()
    x = np.exp(1j * np.arange(cfg.n_beams * cfg.n_range)).reshape(cfg.n_beams, -1) * 1e-3
    a = R.add(x, cfg, 2, -35.0, 1e-10, 5)
    b = R.add(x, cfg, 2, -35.0, 1e-10, 5)
    assert np.array_equal(a, b)
    z = R.add(np.zeros_like(x), cfg, 2, -35.0, 1e-10, 5)
    assert np.allclose(a - x, z, rtol=0, atol=1e-18)
    c = R.add(x, cfg, 3, -35.0, 1e-10, 5)                     # another ping: other samples
    d = R.add(x, cfg, 2, -35.0, 1e-10, 6)                     # another seed
    assert np.abs(c - a).min() > 0 and np.abs(d - a).min() > 0
    # subsets of beams draw the same samples as the full volume
    sub = R.add(x[[3, 40]], cfg, 2, -35.0, 1e-10, 5, beams=[3, 40])
    assert np.array_equal(sub, a[[3, 40]])
