"""FP64 oracle of pulse compression: baseband time series and matched filter.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg. The product package never imports it.

Sec. II-B of the paper asks for time-series data next to the intensity
volumes so that standard processing such as matched filtering can be applied.
The paper fixes neither the pulse nor the sampling, so this oracle takes the
following reading (the GPU path implements the same definitions on its own):

* A beam's complex range column x[n] (the echo volume, one value per range
  bin) is the scene's impulse response sampled at the bins' two-way delay
  spacing dt = 2 dr / c_ref.
* The transmitted baseband pulse is L samples p[0..L-1] at the same spacing.
* Received series:   s[n] = sum_{k=0}^{L-1} p[k] x[n-k],       n in [0, N)
* Matched filter:    y[n] = sum_{k=0}^{L-1} conj(p[k]) s[n+k], n in [0, N)
  with x and s taken as zero outside [0, N) (the record is N samples long).
* Linear-FM pulse of bandwidth B and duration tau: L = max(1, round(tau/dt))
  samples at t_k = (k + 1/2) dt - L dt / 2, p[k] = w[k] exp(i pi (B/tau) t_k^2)
  with w = 1 (rectangular) or w[k] = sin^2(pi (k + 1/2) / L) (Hann).

Every function here is the definition written as loops over pulse taps (no
FFT, no library convolution), in FP64.
"""
from __future__ import annotations

import math

import numpy as np

MAX_TAPS = 64


def lfm_pulse(bandwidth_hz: float, duration_s: float, dt_s: float, window: int = 0) -> np.ndarray:
    """Baseband linear-FM pulse sampled at dt (complex128 [L]); window 0 rect, 1 Hann."""
    if not (bandwidth_hz >= 0.0 and duration_s > 0.0 and dt_s > 0.0) or window not in (0, 1):
        raise ValueError("bandwidth >= 0, duration > 0, dt > 0, window in {0, 1}")
    L = max(1, int(round(duration_s / dt_s)))
    if L > MAX_TAPS:
        raise ValueError(f"pulse of {L} taps; at most {MAX_TAPS}")
    rate = bandwidth_hz / duration_s
    out = np.empty(L, np.complex128)
    for k in range(L):
        t = (k + 0.5) * dt_s - 0.5 * L * dt_s
        w = 1.0 if window == 0 else math.sin(math.pi * (k + 0.5) / L) ** 2
        ph = math.pi * rate * t * t
        out[k] = w * complex(math.cos(ph), math.sin(ph))
    return out


def series(x: np.ndarray, p: np.ndarray) -> np.ndarray:
    """s[b, n] = sum_k p[k] x[b, n - k] over the record [0, N); x is [beams, N]."""
    x = np.asarray(x, np.complex128)
    p = np.asarray(p, np.complex128)
    N = x.shape[-1]
    s = np.zeros_like(x)
    for k in range(min(len(p), N)):
        s[..., k:] += p[k] * x[..., :N - k]
    return s


def matched(s: np.ndarray, p: np.ndarray) -> np.ndarray:
    """y[b, n] = sum_k conj(p[k]) s[b, n + k] over the record [0, N)."""
    s = np.asarray(s, np.complex128)
    p = np.asarray(p, np.complex128)
    N = s.shape[-1]
    y = np.zeros_like(s)
    for k in range(min(len(p), N)):
        y[..., :N - k] += np.conj(p[k]) * s[..., k:]
    return y


def compress(x: np.ndarray, p: np.ndarray):
    """(series, matched) of complex columns x [beams, N] for pulse p."""
    s = series(x, p)
    return s, matched(s, p)
