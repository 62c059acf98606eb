"""Pins of the pulse-compression oracle (time series and matched filter,
Sec. II-B) against shifts of a delta, FFT and library convolutions, the
autocorrelation's symmetry and energy, and closed forms of the linear-FM
pulse (CPU only)."""
import math

import numpy as np
import pytest

from oracle import pulse as P


def _rand(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


@pytest.mark.parametrize("N,L,m", [(50, 7, 0), (50, 7, 20), (50, 7, 46), (5, 9, 2), (1, 3, 0)])
def test_delta_gives_the_pulse(N, L, m):
    p = _rand(L, 1)
    x = np.zeros((1, N), complex)
    x[0, m] = 1.0
    s = P.series(x, p)[0]
    want = np.zeros(N, complex)
    for k in range(L):
        if m + k < N:
            want[m + k] = p[k]
    assert np.array_equal(s, want)


def test_matched_delta_peaks_at_the_delay_with_the_pulse_energy():
    p = P.lfm_pulse(30e3, 400e-6, 19e-6)
    N, m = 200, 90
    x = np.zeros((1, N), complex)
    x[0, m] = 2.0 - 1.0j
    _, y = P.compress(x, p)
    y = y[0]
    energy = float(np.sum(np.abs(p) ** 2))
    assert abs(y[m] - (2.0 - 1.0j) * energy) < 1e-12 * energy
    assert int(np.argmax(np.abs(y))) == m
    L = len(p)
    for j in range(1, L):                         # autocorrelation: R[-j] = conj(R[j])
        assert abs(y[m - j] / (2.0 - 1.0j) - np.conj(y[m + j] / (2.0 - 1.0j))) < 1e-12 * energy
    assert np.all(y[m + L:] == 0) and np.all(y[:m - L + 1] == 0)


def test_series_equals_library_convolution_and_matched_equals_fft_correlation():
    x = _rand((4, 300), 2)
    p = _rand(23, 3)
    s, y = P.compress(x, p)
    N, L = x.shape[1], len(p)
    for b in range(x.shape[0]):
        assert np.allclose(s[b], np.convolve(x[b], p)[:N], rtol=0, atol=1e-12)
    # correlation by FFT of the truncated series (zero beyond the record)
    n = 1 << int(math.ceil(math.log2(N + L)))
    S = np.fft.fft(s, n, axis=1)
    Pp = np.fft.fft(p, n)
    corr = np.fft.ifft(S * np.conj(Pp)[None, :], axis=1)[:, :N]
    assert np.allclose(y, corr, rtol=0, atol=1e-10)


def test_linear_and_shift_invariant():
    p = _rand(11, 4)
    a, b = 0.7 - 0.2j, -1.3 + 0.5j
    x1, x2 = _rand((2, 120), 5), _rand((2, 120), 6)
    s1, y1 = P.compress(x1, p)
    s2, y2 = P.compress(x2, p)
    s, y = P.compress(a * x1 + b * x2, p)
    assert np.allclose(s, a * s1 + b * s2, atol=1e-12) and np.allclose(y, a * y1 + b * y2, atol=1e-12)
    # shift: an input confined to the middle of the record moves its outputs rigidly
    x = np.zeros((1, 200), complex)
    x[0, 60:80] = _rand(20, 7)
    sa, ya = P.compress(x, p)
    sb, yb = P.compress(np.roll(x, 37, axis=1), p)
    assert np.allclose(np.roll(sa, 37, axis=1), sb, atol=1e-12)
    assert np.allclose(np.roll(ya, 37, axis=1), yb, atol=1e-12)


def test_single_tap_pulse_scales():
    c = 0.6 + 0.8j
    x = _rand((3, 17), 8)
    s, y = P.compress(x, np.array([c]))
    assert np.allclose(s, c * x, atol=1e-15) and np.allclose(y, abs(c) ** 2 * x, atol=1e-15)


def test_lfm_pulse_closed_forms():
    B, tau, dt = 40e3, 300e-6, 300e-6 / 16
    p = P.lfm_pulse(B, tau, dt)
    L = len(p)
    assert L == 16
    assert np.allclose(np.abs(p), 1.0, atol=1e-15)
    assert np.allclose(p, p[::-1], atol=1e-15)                     # even phase about the centre
    ph = np.unwrap(np.angle(p))
    d2 = np.diff(ph, 2)                                             # quadratic phase: constant second difference
    assert np.allclose(d2, 2.0 * math.pi * (B / tau) * dt * dt, atol=1e-12)
    h = P.lfm_pulse(B, tau, dt, window=1)
    assert abs(np.sum(np.abs(h)) - L / 2) < 1e-12                   # sum of sin^2 over the L cells is L / 2
    assert np.allclose(np.abs(h), np.sin(math.pi * (np.arange(L) + 0.5) / L) ** 2, atol=1e-15)
    with pytest.raises(ValueError):
        P.lfm_pulse(B, 65 * dt, dt)


@pytest.mark.parametrize("window,lo,hi", [(0, -14.5, -12.0), (1, -60.0, -25.0)])
def test_lfm_matched_response_mainlobe_and_sidelobes(window, lo, hi):
    """Large time-bandwidth LFM: the compressed mainlobe's first nulls sit
    about 1/B from the peak, and the peak sidelobe is near the sinc value
    (-13.3 dB) for a rectangular envelope and far lower with a Hann one."""
    dt = 1.0
    B, tau = 0.4, 64.0                         # 2.5 samples per resolution cell, TB = 25.6
    p = P.lfm_pulse(B, tau, dt, window)
    N, m = 400, 200
    x = np.zeros((1, N), complex)
    x[0, m] = 1.0
    _, y = P.compress(x, p)
    a = np.abs(y[0]) / np.abs(y[0, m])
    # first local minimum right of the peak
    j = m + 1
    while a[j + 1] < a[j]:
        j += 1
    if window == 0:
        assert abs((j - m) - 1.0 / (B * dt)) <= 1.0
    side = 20 * math.log10(max(a[j:m + len(p)].max(), 1e-300))
    assert lo <= side <= hi, side
