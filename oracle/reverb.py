"""FP64 oracle of water-column volume reverberation and receiver noise.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg. The product package never imports it.

Sec. II-B names, as extensions, scattering from within the water volume
and speckle. It gives no model, so this
oracle takes the following reading (the GPU path implements the same
definition on its own):

* Every range cell (beam b = v * n_h + h, bin n) of cell-centred beams holds
  many unresolved scatterers, so its summed echo is a circular complex
  Gaussian (fully developed speckle) with mean power
      P(b, n) = s_v * V / r^4 * 10^(-alpha * 2 r / 10) + N0,
  r = r_min + (n + 1/2) dr the bin centre, V = r^2 cos(el_v) dth_h dth_v dr
  the cell's volume (el_v its centre elevation), s_v = 10^(S_v / 10) the
  volume scattering coefficient (1/m) and N0 the receiver noise power per
  cell. Spreading and absorption are those of the echo model (two-way).
* The sample is E += sqrt(P / 2) * (g1 + i g2) with (g1, g2) from the
  Box-Muller transform of two uniforms drawn by the counter-based SplitMix64
  generator: z = splitmix64(seed, c + 1) with counter
  c = (ping << 43) xor (b << 12) xor n; u1 = ((z >> 40) + 1) / 2^24,
  u2 = ((z >> 16) mod 2^24) / 2^24; g1 + i g2 = sqrt(-2 ln u1) e^(2 pi i u2).
* No shadowing: the water column behind the first surface is insonified too.

SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) is written out here in numpy
from its published definition, vectorised over counters.
"""
from __future__ import annotations

import math

import numpy as np

_GOLD = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n) -> np.ndarray:
    """The n-th output (n >= 1) of SplitMix64 started at `seed`, for an array of n."""
    n = np.asarray(n, np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + n * _GOLD
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def counters(ping: int, beams, bins) -> np.ndarray:
    b = np.asarray(beams, np.uint64)[:, None]
    n = np.asarray(bins, np.uint64)[None, :]
    return (np.uint64(ping) << np.uint64(43)) ^ (b << np.uint64(12)) ^ n


def gaussians(seed: int, ping: int, beams, bins) -> np.ndarray:
    """Complex standard-normal pairs g1 + i g2 per (beam, bin), complex128."""
    z = splitmix64(seed, counters(ping, beams, bins) + np.uint64(1))
    u1 = ((z >> np.uint64(40)).astype(np.float64) + 1.0) / 16777216.0
    u2 = ((z >> np.uint64(16)) & np.uint64(0xFFFFFF)).astype(np.float64) / 16777216.0
    rad = np.sqrt(-2.0 * np.log(u1))
    return rad * np.cos(2.0 * math.pi * u2) + 1j * rad * np.sin(2.0 * math.pi * u2)


def mean_power(cfg, beams, bins, sv_db: float, noise_power: float) -> np.ndarray:
    """P(b, n) for the listed beams and bins of a ping layout ``cfg``."""
    beams = np.asarray(beams, np.int64)
    bins = np.asarray(bins, np.int64)
    dh, dv = cfg.hfov / cfg.n_h, cfg.vfov / cfg.n_v
    dr = (cfg.r_max - cfg.r_min) / cfg.n_range
    r = cfg.r_min + (bins + 0.5) * dr
    el = -0.5 * cfg.vfov + (beams // cfg.n_h + 0.5) * dv
    sv = 10.0 ** (sv_db / 10.0)
    vol = (r[None, :] ** 2) * np.cos(el)[:, None] * dh * dv * dr
    return sv * vol / r[None, :] ** 4 * 10.0 ** (-cfg.abs_db_per_m * 2.0 * r[None, :] / 10.0) + noise_power


def add(volume, cfg, ping: int, sv_db: float, noise_power: float, seed: int, beams=None) -> np.ndarray:
    """volume [beams, n_bins] (the listed beams, all by default) plus the
    reverberation-and-noise sample of every cell, complex128."""
    volume = np.asarray(volume, np.complex128)
    nb = volume.shape[0]
    beams = np.arange(nb) if beams is None else np.asarray(beams, np.int64)
    bins = np.arange(volume.shape[1])
    P = mean_power(cfg, beams, bins, sv_db, noise_power)
    return volume + np.sqrt(P / 2.0) * gaussians(seed, ping, beams, bins)
