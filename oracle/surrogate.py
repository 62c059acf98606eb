"""FP64 NumPy oracle of the learned multipath surrogate.

TEST INFRASTRUCTURE ONLY: used by tests/ and the benchmark's baseline leg,
never by the product path. It shares no code with the HIP kernels.

The paper (Sec. II-B) allows scattering functions to be learned from data;
here a small network predicts, from each beam's single-bounce G-buffer, the
range profile that further bounces add, as the dB residual between the
incoherent multi-bounce and single-bounce intensity, compressed to the first
64 coefficients of an orthonormal DCT-II of the 1,024-bin profile.

Network (168,768 parameters): a 3 x 3 beam-neighbourhood convolution of the
7 G-buffer features (written as an im2col product with 63 inputs, zero
padding at the edges) -> ReLU -> 64 -> 256 -> 256 -> 256 -> 64 dense layers
with ReLU between them. Loss: mean squared error over the 64 standardised
coefficients.

Parameter vector layout (float, 168,768 entries): for each layer in order
W [K][N] row-major then b [N], with (K, N) = (63, 64), (64, 256), (256, 256),
(256, 256), (256, 64).
"""
from __future__ import annotations

import numpy as np

LAYERS = ((63, 64), (64, 256), (256, 256), (256, 256), (256, 64))
N_FEAT = 7
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


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (the random draws are inputs to both sides)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for k, n in LAYERS:
        lim = np.sqrt(6.0 / k)
        parts.append(rng.uniform(-lim, lim, k * n))
        parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


def im2col(gbuf):
    """gbuf [n_img, H, W, >= 7] -> [n_img * H * W, 63]: for each beam (v, h)
    the 7 features of (v + dv, h + dh), dv, dh in {-1, 0, 1}, zero outside,
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


def forward(theta, x0):
    """Returns (activations [x0 .. x4], y): x_{l+1} = relu(x_l W_l + b_l), y = x4 W4 + b4."""
    L = unpack(theta)
    acts = [np.asarray(x0, np.float64)]
    x = acts[0]
    for i, (W, b) in enumerate(L):
        z = x @ W + b
        if i < len(L) - 1:
            x = np.maximum(z, 0.0)
            acts.append(x)
        else:
            return acts, z
    raise AssertionError


def mse(y, t):
    d = y - np.asarray(t, np.float64)
    return float((d * d).mean()), 2.0 * d / d.size


def backward(theta, acts, dy):
    """Gradient of the loss w.r.t. the flat parameter vector, given dL/dy."""
    L = unpack(theta)
    grads = [None] * len(L)
    dz = dy
    for i in range(len(L) - 1, -1, -1):
        W, _ = L[i]
        x = acts[i]
        grads[i] = (x.T @ dz, dz.sum(axis=0))
        if i > 0:
            dx = dz @ W.T
            dz = dx * (acts[i] > 0.0)
    return pack(grads)


def loss_and_grad(theta, gbuf, target):
    acts, y = forward(theta, im2col(gbuf))
    loss, dy = mse(y, target)
    return loss, backward(theta, acts, dy), y


def dct_basis(n_bins: int, n_coef: int = N_COEF):
    """Orthonormal DCT-II basis [n_coef, n_bins]:
    C[k, r] = s_k cos(pi (r + 1/2) k / n_bins), s_0 = sqrt(1/n), s_k = sqrt(2/n)."""
    r = np.arange(n_bins) + 0.5
    k = np.arange(n_coef)[:, None]
    C = np.cos(np.pi * r[None, :] * k / n_bins)
    C *= np.sqrt(2.0 / n_bins)
    C[0] *= np.sqrt(0.5)
    return C


def residual_db(i1, im, floor=I_FLOOR):
    """dB residual of the multi-bounce incoherent profile over the single-bounce one."""
    i1 = np.asarray(i1, np.float64)
    im = np.asarray(im, np.float64)
    return 10.0 * np.log10(i1 + im + floor) - 10.0 * np.log10(i1 + floor)


def residual_coefficients(i1, im, floor=I_FLOOR):
    """[rows, n_bins] incoherent channels -> [rows, 64] DCT coefficients of the residual."""
    res = residual_db(i1, im, floor)
    return res @ dct_basis(res.shape[-1]).T


def profile_from_coefficients(i1, coef, floor=I_FLOOR):
    """Predicted multi-bounce dB profile: single-bounce dB + inverse DCT of the coefficients."""
    i1 = np.asarray(i1, np.float64)
    return 10.0 * np.log10(i1 + floor) + np.asarray(coef, np.float64) @ dct_basis(i1.shape[-1])


def beam_errors(i1, im, pred_profile, floor=I_FLOOR, occupied_db=3.0):
    """Mean |pred - truth| in dB per beam over occupied bins (truth more than
    `occupied_db` above the floor); NaN for beams with none."""
    truth = 10.0 * np.log10(np.asarray(i1, np.float64) + np.asarray(im, np.float64) + floor)
    occ = truth > 10.0 * np.log10(floor) + occupied_db
    err = np.abs(np.asarray(pred_profile, np.float64) - truth)
    n = occ.sum(axis=-1)
    with np.errstate(invalid="ignore"):
        return np.where(n > 0, (err * occ).sum(axis=-1) / np.maximum(n, 1), np.nan), n
