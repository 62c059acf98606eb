"""FP64 NumPy oracle of the learned multipath surrogate.

TEST INFRASTRUCTURE ONLY: used by tests/ and the benchmark's baseline leg,
never by the product path. It shares no code with the HIP kernels.

The paper (Sec. II-B) allows scattering functions to be learned from data;
here a small network predicts, from each beam's single-bounce G-buffer, the
range profile that further bounces add: the dB level of the later-bounce
incoherent intensity above the intensity floor, 10 log10(1 + Im / floor),
range-smoothed, shifted to start at the beam's first-hit bin and compressed
to the first 64 coefficients of an orthonormal DCT-II of the 1,024-bin
profile. The predicted multi-bounce profile adds that intensity back to the
single-bounce one: 10 log10(I1 + floor 10^(q / 10)), so a zero prediction is
the single-bounce profile.

Network input per beam: a 3 x 3 beam-neighbourhood convolution of the 8
G-buffer features (the first-hit statistics and the beam axis's vertical
component; written as an im2col product with 72 inputs, zero padding at the
edges), followed by the beam's geometry (geometry_features): where its mean
first hit lies in the world, the beam axis in the world, the sensor
position and the axis mirrored at the mean first-hit normal (the direction
a specular continuation takes), plus sines and cosines of all but the
sensor position at N_FREQ octaves. Later bounces go where the scene sends
the continuation of that first hit, so the network of one scene needs to
know where in the scene the hit is and where it sends the continuation.

Network: input -> 64 -> 256 -> 256 -> 256 -> 64 dense layers with ReLU
between them. Loss: mean squared error over the 64 standardised
coefficients, coefficient j weighted by w_j (by default 1; in training
sigma_j^2 / mean(sigma^2), which makes it the squared error of the profile
itself by Parseval's theorem).

Parameter vector layout (float, param_count() entries): for each layer in
order W [K][N] row-major then b [N], with (K, N) = (N_IN, 64), (64, 256),
(256, 256), (256, 256), (256, 64).
"""
from __future__ import annotations

import numpy as np

N_FEAT = 8
N_FREQ = 5                       # octaves of the geometry's sines and cosines
N_GEO = 12 + 18 * N_FREQ         # geometry features per beam
N_IN = 9 * N_FEAT + N_GEO        # network inputs per beam
GEO_STRIDE = 16                  # floats of one image's geometry block
LAYERS = ((N_IN, 64), (64, 256), (256, 256), (256, 256), (256, 64))
N_COEF = 64
I_FLOOR = 1e-11


def param_count() -> int:
    return sum(k * n + n for k, n in LAYERS)


def unpack(theta):
    """Flat parameter vector -> list of (W [K, N], b [N])."""
    out, o = [], 0
    for k, n in LAYERS:
        W = np.asarray(theta[o:o + k * n], np.float64).reshape(k, n)
        o += k * n
        b = np.asarray(theta[o:o + n], np.float64)
        o += n
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def im2col(gbuf):
    """gbuf [n_img, H, W, 8] -> [n_img * H * W, 72]: for each beam (v, h)
    the 8 features of (v + dv, h + dh), dv, dh in {-1, 0, 1}, zero outside,
    ordered (dv, dh, feature)."""
    g = np.asarray(gbuf, np.float64)[..., :N_FEAT]
    n, H, W, _ = g.shape
    pad = np.zeros((n, H + 2, W + 2, N_FEAT))
    pad[:, 1:-1, 1:-1] = g
    cols = []
    for dv in (-1, 0, 1):
        for dh in (-1, 0, 1):
            cols.append(pad[:, 1 + dv:1 + dv + H, 1 + dh:1 + dh + W])
    return np.concatenate(cols, axis=-1).reshape(n * H * W, 9 * N_FEAT)


def geometry_block(position, rot, hfov, vfov):
    """One image's geometry block (GEO_STRIDE floats): sensor position (3),
    the sensor-to-world rotation row-major (9), the horizontal and vertical
    fields of view, two zeros."""
    g = np.zeros(GEO_STRIDE)
    g[0:3] = np.asarray(position, np.float64)
    g[3:12] = np.asarray(rot, np.float64).reshape(9)
    g[12], g[13] = hfov, vfov
    return g


def geometry_features(gbuf, geo, r_max):
    """gbuf [n_img, H, W, 8], geo [n_img, GEO_STRIDE] -> [n_img * H * W, N_GEO].

    Beam (v, h) of a cell-centred H x W layout has its axis at azimuth
    -hfov/2 + (h + 1/2) hfov / W and elevation -vfov/2 + (v + 1/2) vfov / H,
    the unit vector (cos el cos az, cos el sin az, sin el) in the sensor
    frame, u = R times it in the world. Its mean first hit is taken on that
    axis at the G-buffer's mean range: P = S + r_max g0 u when the beam has a
    hit (g6 > 0), else the origin. The mirror direction reflects u at the
    mean first-hit normal n = (g3, g4, g5) (the law of specular reflection,
    for a normal of any length): m = u - 2 (u . n) n / (n . n), zero without
    a hit or with a zero normal. Features, in metres / 10 and unit vectors:
    P / 10 (3), u (3), S / 10 (3), m (3), then sin(pi/2 2^k x) for x in
    (P / 10, u, m) and k = 0 .. N_FREQ - 1 (x-major), then the cosines in the
    same order."""
    g = np.asarray(gbuf, np.float64)
    n, H, W, _ = g.shape
    out = np.zeros((n, H, W, N_GEO))
    for i in range(n):
        S = np.asarray(geo[i][0:3], np.float64)
        R = np.asarray(geo[i][3:12], np.float64).reshape(3, 3)
        hfov, vfov = float(geo[i][12]), float(geo[i][13])
        for v in range(H):
            el = -0.5 * vfov + (v + 0.5) * vfov / H
            for h in range(W):
                az = -0.5 * hfov + (h + 0.5) * hfov / W
                us = np.array([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])
                u = R @ us
                hit = g[i, v, h, 6] > 0
                P = S + r_max * g[i, v, h, 0] * u if hit else np.zeros(3)
                nrm = g[i, v, h, 3:6]
                nn = float(nrm @ nrm)
                m = u - 2.0 * float(u @ nrm) / nn * nrm if (hit and nn > 1e-12) else np.zeros(3)
                x = np.concatenate([P / 10.0, u, m])
                arg = np.array([[np.pi / 2.0 * 2.0 ** k * xx for k in range(N_FREQ)] for xx in x])
                out[i, v, h] = np.concatenate([P / 10.0, u, S / 10.0, m, np.sin(arg).reshape(-1),
                                               np.cos(arg).reshape(-1)])
    return out.reshape(n * H * W, N_GEO)


def inputs(gbuf, geo, r_max):
    """Network input rows [n_img * H * W, N_IN]: im2col of the G-buffer, then the geometry."""
    return np.concatenate([im2col(gbuf), geometry_features(gbuf, geo, r_max)], axis=1)


def forward(theta, x0, store=None):
    """Returns (activations [x0 .. x4], y): x_{l+1} = relu(x_l W_l + b_l), y = x4 W4 + b4.
    `store`, if given, is applied to every stored activation (a test hook that
    models a lower storage precision; by default values are kept exact)."""
    st = store if store is not None else (lambda a: a)
    L = unpack(theta)
    acts = [st(np.asarray(x0, np.float64))]
    x = acts[0]
    for i, (W, b) in enumerate(L):
        z = x @ W + b
        if i < len(L) - 1:
            x = st(np.maximum(z, 0.0))
            acts.append(x)
        else:
            return acts, z
    raise AssertionError


def mse(y, t, w=None):
    """Weighted mean squared error sum_j w_j (y - t)^2 / (rows * 64) and its
    gradient with respect to y (w None: all weights 1)."""
    d = y - np.asarray(t, np.float64)
    wj = np.ones(d.shape[-1]) if w is None else np.asarray(w, np.float64)
    return float((wj * d * d).mean()), 2.0 * wj * d / d.size


def backward(theta, acts, dy, store=None):
    """Gradient of the loss w.r.t. the flat parameter vector, given dL/dy.
    `store` as in forward(), applied to every stored layer gradient."""
    st = store if store is not None else (lambda a: a)
    L = unpack(theta)
    grads = [None] * len(L)
    dz = st(dy)
    for i in range(len(L) - 1, -1, -1):
        W, _ = L[i]
        x = acts[i]
        grads[i] = (x.T @ dz, dz.sum(axis=0))
        if i > 0:
            dx = dz @ W.T
            dz = st(dx * (acts[i] > 0.0))
    return pack(grads)


def loss_and_grad(theta, x0, target, store=None, w=None):
    """Loss, parameter gradient and output for input rows x0 (inputs())."""
    acts, y = forward(theta, x0, store)
    loss, dy = mse(y, target, w)
    return loss, backward(theta, acts, dy, store), y


def dct_basis(n_bins: int, n_coef: int = N_COEF):
    """Orthonormal DCT-II basis [n_coef, n_bins]:
    C[k, r] = s_k cos(pi (r + 1/2) k / n_bins), s_0 = sqrt(1/n), s_k = sqrt(2/n)."""
    r = np.arange(n_bins) + 0.5
    k = np.arange(n_coef)[:, None]
    C = np.cos(np.pi * r[None, :] * k / n_bins)
    C *= np.sqrt(2.0 / n_bins)
    C[0] *= np.sqrt(0.5)
    return C


SMOOTH = 32     # range smoothing of the incoherent intensities (bins)


def smooth_range(a, w=SMOOTH):
    """Box average over bins [r - w/2, r + w/2) along the last axis, zero outside."""
    a = np.asarray(a, np.float64)
    n = a.shape[-1]
    out = np.zeros_like(a)
    for r in range(n):
        lo, hi = max(0, r - w // 2), min(n, r + w - w // 2)
        out[..., r] = a[..., lo:hi].sum(axis=-1) / w
    return out


def first_hit_bin(gbuf_rows, r_min, r_max, n_bins):
    """Range bin of each beam's mean first-bounce range (G-buffer feature 0 is
    range / r_max, feature 6 the hit fraction); 0 for beams without hits."""
    g = np.asarray(gbuf_rows, np.float32)
    dr = np.float32((r_max - r_min) / n_bins)
    R = g[:, 0] * np.float32(r_max)
    b = np.floor((R - np.float32(r_min)) / dr)
    b = np.where(g[:, 6] > 0, b, 0)
    return np.clip(b, 0, n_bins - 1).astype(np.int64)


def level_db(im, floor=I_FLOOR):
    """dB level of the later-bounce intensity above the floor: 10 log10(1 + Im / floor)."""
    return 10.0 * np.log10(1.0 + np.asarray(im, np.float64) / floor)


def level_coefficients(im, floor=I_FLOOR):
    """[rows, n_bins] later-bounce channel -> [rows, 64] DCT coefficients of its level."""
    lv = level_db(im, floor)
    return lv @ dct_basis(lv.shape[-1]).T


def profile_from_coefficients(i1, coef, floor=I_FLOOR):
    """Predicted multi-bounce dB profile: the single-bounce intensity plus the
    later-bounce intensity of the level the coefficients give."""
    i1 = np.asarray(i1, np.float64)
    q = np.asarray(coef, np.float64) @ dct_basis(i1.shape[-1])
    return 10.0 * np.log10(i1 + floor * 10.0 ** (q / 10.0))


def aligned_level_coefficients(im, r1, floor=I_FLOOR, w=SMOOTH):
    """DCT coefficients of the range-smoothed later-bounce level shifted so that
    each beam's first-hit bin r1 becomes bin 0 (bins past the end are zero)."""
    lv = level_db(smooth_range(im, w), floor)
    n = lv.shape[-1]
    al = np.zeros_like(lv)
    for q in range(lv.shape[0]):
        al[q, :n - r1[q]] = lv[q, r1[q]:]
    return al @ dct_basis(n).T


def aligned_level(coef, r1, n):
    """[rows, n] level profile: the inverse DCT of the coefficients shifted
    back to start at each beam's first-hit bin (level 0 before it)."""
    q = np.asarray(coef, np.float64) @ dct_basis(n)
    lv = np.zeros((q.shape[0], n))
    for k in range(lv.shape[0]):
        lv[k, r1[k]:] = q[k, :n - r1[k]]
    return lv


def aligned_profile(i1, coef, r1, floor=I_FLOOR, w=SMOOTH):
    """Predicted range-smoothed multi-bounce dB profile: the smoothed
    single-bounce intensity plus the later-bounce intensity of the level."""
    i1s = smooth_range(i1, w)
    lv = aligned_level(coef, r1, i1s.shape[-1])
    return 10.0 * np.log10(i1s + floor * 10.0 ** (lv / 10.0))


def full_profile(i1, coef, r1, floor=I_FLOOR):
    """Predicted multi-bounce dB profile at full range resolution: the raw
    single-bounce intensity plus the later-bounce intensity of the level."""
    i1 = np.asarray(i1, np.float64)
    lv = aligned_level(coef, r1, i1.shape[-1])
    return 10.0 * np.log10(i1 + floor * 10.0 ** (lv / 10.0))


def aligned_beam_errors(i1, im, pred_profile, floor=I_FLOOR, occupied_db=3.0, w=SMOOTH):
    """beam_errors() against the range-smoothed truth."""
    return beam_errors(smooth_range(i1, w), smooth_range(im, w), pred_profile, floor, occupied_db)


def beam_errors(i1, im, pred_profile, floor=I_FLOOR, occupied_db=3.0):
    """Mean |pred - truth| in dB per beam over occupied bins (truth more than
    `occupied_db` above the floor); NaN for beams with none."""
    truth = 10.0 * np.log10(np.asarray(i1, np.float64) + np.asarray(im, np.float64) + floor)
    occ = truth > 10.0 * np.log10(floor) + occupied_db
    err = np.abs(np.asarray(pred_profile, np.float64) - truth)
    n = occ.sum(axis=-1)
    with np.errstate(invalid="ignore"):
        return np.where(n > 0, (err * occ).sum(axis=-1) / np.maximum(n, 1), np.nan), n
