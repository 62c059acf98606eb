"""Pins of the FP64 surrogate oracle: finite differences, the DCT against the
library routine and its orthonormality, im2col by brute force."""
import numpy as np
import pytest
from scipy import fft

from oracle import surrogate as SO
from paper_2606_06130_amd.scenes import surrogate_init_params


def test_parameter_count():
    # (72 neighbourhood + 102 geometry inputs) x 64, then 64 x 256, 2 x 256 x 256 and 256 x 64, with biases
    assert SO.N_IN == 174 and SO.N_GEO == 102
    assert SO.param_count() == 174 * 64 + 64 + 64 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 64 + 64 == 175872


def _rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def _geo_cols(f):
    """Split geometry columns: P/10, u, S/10, sines [9, N_FREQ], cosines [9, N_FREQ] (the mirror
    direction m is _mirror(f))."""
    F = SO.N_FREQ
    return (f[:, 0:3], f[:, 3:6], f[:, 6:9], f[:, 12:12 + 9 * F].reshape(-1, 9, F),
            f[:, 12 + 9 * F:].reshape(-1, 9, F))


def _mirror(f):
    return f[:, 9:12]


def test_geometry_axis_hit_point_and_rotation():
    """The centre beam of a 1 x 1 layout looks along the sensor's x axis: with
    a 90-degree yaw that is the world y axis, and the mean first hit lies on
    it at the G-buffer range; a sensor pitched down by a leaves it with
    vertical component -sin a."""
    S = np.array([1.0, -2.0, -3.0])
    g = np.zeros((1, 1, 1, 8))
    g[..., 0] = 0.4
    g[..., 6] = 1.0
    f = SO.geometry_features(g, [SO.geometry_block(S, _rot_z(np.pi / 2), 0.3, 0.2)], 15.0)
    P10, u, S10, _, _ = _geo_cols(f)
    np.testing.assert_allclose(u[0], [0.0, 1.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(P10[0] * 10.0, S + np.array([0.0, 6.0, 0.0]), atol=1e-12)
    np.testing.assert_allclose(S10[0] * 10.0, S, atol=1e-15)
    a = 0.35
    f = SO.geometry_features(g, [SO.geometry_block(S, _rot_y(a), 0.3, 0.2)], 15.0)
    _, u, _, _, _ = _geo_cols(f)
    np.testing.assert_allclose(u[0], [np.cos(a), 0.0, -np.sin(a)], atol=1e-15)


def test_geometry_layout_symmetry_and_range():
    """Cell-centred beams of a 2 x 2 layout: opposite corners mirror in the
    sensor's y and z, each axis is a unit vector, and P - S is the axis times
    the G-buffer range; a beam without a hit has P at the origin."""
    rng = np.random.Generator(np.random.PCG64(9))
    g = np.zeros((1, 2, 2, 8))
    g[..., 0] = rng.uniform(0.1, 0.9, (1, 2, 2))
    g[..., 6] = 1.0
    g[0, 1, 0, 6] = 0.0                                    # no hit in beam (v=1, h=0)
    S = rng.normal(size=3)
    f = SO.geometry_features(g, [SO.geometry_block(S, np.eye(3), 0.8, 0.6)], 15.0)
    P10, u, _, _, _ = _geo_cols(f)
    np.testing.assert_allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-15)
    # rows are (v, h) = (0,0), (0,1), (1,0), (1,1): (0,0) and (1,1) mirror in y and z
    np.testing.assert_allclose(u[0] * [1, -1, -1], u[3], atol=1e-15)
    np.testing.assert_allclose(u[1] * [1, -1, -1], u[2], atol=1e-15)
    assert u[0, 1] < 0 and u[0, 2] < 0                    # h = 0 looks right (-y), v = 0 looks down
    for row, v, h in ((0, 0, 0), (1, 0, 1), (3, 1, 1)):
        np.testing.assert_allclose(P10[row] * 10.0 - S, 15.0 * g[0, v, h, 0] * u[row], atol=1e-12)
    np.testing.assert_array_equal(P10[2], 0.0)


def test_geometry_fourier_columns():
    """Sines and cosines at octaves: sin^2 + cos^2 = 1, each octave's sine is
    the double angle of the one below (sin 2t = 2 sin t cos t), the lowest
    octave is a quarter turn per unit, and a zero input gives (0, 1)."""
    rng = np.random.Generator(np.random.PCG64(10))
    g = np.zeros((2, 3, 4, 8))
    g[..., 0] = rng.uniform(0.05, 1.0, (2, 3, 4))
    g[..., 6] = rng.random((2, 3, 4)) < 0.7
    geo = [SO.geometry_block(rng.normal(size=3) * 5, _rot_z(rng.uniform(-3, 3)) @ _rot_y(rng.uniform(-1, 1)), 1.2, 0.5)
           for _ in range(2)]
    f = SO.geometry_features(g, geo, 15.0)
    P10, u, _, sn, cs = _geo_cols(f)
    x = np.concatenate([P10, u, _mirror(f)], axis=1)
    np.testing.assert_allclose(sn ** 2 + cs ** 2, 1.0, atol=1e-14)
    np.testing.assert_allclose(sn[:, :, 0], np.sin(np.pi / 2 * x), atol=1e-14)
    for k in range(1, SO.N_FREQ):
        np.testing.assert_allclose(sn[:, :, k], 2 * sn[:, :, k - 1] * cs[:, :, k - 1], atol=1e-13)
        np.testing.assert_allclose(cs[:, :, k], cs[:, :, k - 1] ** 2 - sn[:, :, k - 1] ** 2, atol=1e-13)
    nohit = (g[..., 6] <= 0).reshape(-1)
    assert nohit.any()
    np.testing.assert_array_equal(sn[nohit, :3], 0.0)
    np.testing.assert_array_equal(cs[nohit, :3], 1.0)
    np.testing.assert_array_equal(sn[nohit, 6:], 0.0)
    np.testing.assert_array_equal(cs[nohit, 6:], 1.0)


def test_geometry_mirror_direction():
    """The mirror direction is the law of reflection at the mean first-hit
    normal: a horizontal seabed (normal +z) flips the vertical component, a
    wall facing -x flips the x component; the normal's length and sign do not
    matter; the mirror is a unit vector at the same angle to the normal as
    the axis, mirroring it back gives the axis, and it is zero for a beam
    without a hit or without a normal."""
    rng = np.random.Generator(np.random.PCG64(12))
    S = np.array([0.5, -1.0, -3.0])
    geo = [SO.geometry_block(S, _rot_z(0.3) @ _rot_y(0.6), 1.0, 0.5)]
    g = np.zeros((1, 2, 3, 8))
    g[..., 0] = 0.3
    g[..., 6] = 1.0
    g[0, 0, 0, 3:6] = [0.0, 0.0, 1.0]                  # seabed
    g[0, 0, 1, 3:6] = [-0.4, 0.0, 0.0]                 # wall facing -x, normal of length 0.4
    g[0, 0, 2, 3:6] = [0.0, 0.0, -2.0]                 # seabed normal, opposite sign and length 2
    g[0, 1, 0, 3:6] = rng.normal(size=3)               # any surface
    g[0, 1, 1, 6] = 0.0                                # no hit
    g[0, 1, 1, 3:6] = [0.0, 0.0, 1.0]
    g[0, 1, 2, 3:6] = 0.0                              # a hit without a normal
    f = SO.geometry_features(g, geo, 15.0)
    _, u, _, _, _ = _geo_cols(f)
    m = _mirror(f)
    np.testing.assert_allclose(m[0], u[0] * [1, 1, -1], atol=1e-15)
    np.testing.assert_allclose(m[1], u[1] * [-1, 1, 1], atol=1e-15)
    np.testing.assert_allclose(m[2], u[2] * [1, 1, -1], atol=1e-15)
    n = g[0, 1, 0, 3:6] / np.linalg.norm(g[0, 1, 0, 3:6])
    assert abs(np.linalg.norm(m[3]) - 1.0) < 1e-14
    assert abs(m[3] @ n + u[3] @ n) < 1e-14            # same angle, other side
    np.testing.assert_allclose(m[3] - u[3], -2.0 * (u[3] @ n) * n, atol=1e-14)   # the change lies along the normal
    np.testing.assert_allclose(m[3] - 2.0 * (m[3] @ n) * n, u[3], atol=1e-14)    # mirroring back gives the axis
    np.testing.assert_array_equal(m[4], 0.0)
    np.testing.assert_array_equal(m[5], 0.0)


def test_inputs_concatenate_im2col_and_geometry():
    rng = np.random.Generator(np.random.PCG64(11))
    g = rng.normal(size=(1, 3, 5, 8))
    geo = [SO.geometry_block([0.0, 1.0, 2.0], np.eye(3), 1.0, 0.4)]
    x = SO.inputs(g, geo, 15.0)
    assert x.shape == (15, SO.N_IN)
    np.testing.assert_array_equal(x[:, :72], SO.im2col(g))
    np.testing.assert_array_equal(x[:, 72:], SO.geometry_features(g, geo, 15.0))


def test_im2col_brute_force():
    rng = np.random.Generator(np.random.PCG64(1))
    g = rng.normal(size=(2, 5, 6, 8))
    X = SO.im2col(g)
    assert X.shape == (60, 72)
    for n in range(2):
        for v in range(5):
            for h in range(6):
                row = X[n * 30 + v * 6 + h]
                q = 0
                for dv in (-1, 0, 1):
                    for dh in (-1, 0, 1):
                        vv, hh = v + dv, h + dh
                        want = g[n, vv, hh, :8] if 0 <= vv < 5 and 0 <= hh < 6 else np.zeros(8)
                        np.testing.assert_array_equal(row[q:q + 8], want)
                        q += 8


@pytest.mark.parametrize("weighted", [False, True])
def test_gradients_match_central_differences(weighted):
    rng = np.random.Generator(np.random.PCG64(2))
    theta = surrogate_init_params(3).astype(np.float64)
    theta += rng.normal(0, 0.01, theta.size)                  # nonzero biases
    g = rng.uniform(-1, 1, size=(1, 4, 5, 8))
    x0 = SO.inputs(g, [SO.geometry_block(rng.normal(size=3), _rot_z(0.7), 1.0, 0.5)], 15.0)
    t = rng.normal(size=(20, 64))
    w = rng.uniform(0.1, 3.0, 64) if weighted else None
    loss, grad, _ = SO.loss_and_grad(theta, x0, t, w=w)
    idx = rng.choice(theta.size, 60, replace=False)
    # include entries of every layer's weights and biases
    offs = np.cumsum([0] + [k * n + n for k, n in SO.LAYERS])
    for a, b in zip(offs[:-1], offs[1:]):
        idx = np.concatenate([idx, [a, b - 1]])
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        lp = SO.loss_and_grad(tp, x0, t, w=w)[0]
        lm = SO.loss_and_grad(tm, x0, t, w=w)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, grad[i])


def test_dct_matches_library_and_is_orthonormal():
    n = 1024
    C = SO.dct_basis(n, n)
    x = np.random.Generator(np.random.PCG64(4)).normal(size=(3, n))
    np.testing.assert_allclose(x @ C.T, fft.dct(x, type=2, norm="ortho", axis=-1), atol=1e-12)
    np.testing.assert_allclose(C @ C.T, np.eye(n), atol=1e-12)           # orthonormal -> IDCT(DCT(x)) = x
    np.testing.assert_allclose((x @ C.T) @ C, x, atol=1e-12)
    c = x @ C.T
    np.testing.assert_allclose((c ** 2).sum(-1), (x ** 2).sum(-1), rtol=1e-12)   # Parseval
    e = np.zeros(n)
    e[5] = 1.0
    np.testing.assert_allclose(e @ C, C[5])                               # a basis vector maps back
    np.testing.assert_allclose(C[5] @ C.T, e, atol=1e-12)                  # and to a delta


def test_truncated_profile_is_projection():
    """The predicted profile from the 64 level coefficients adds back the
    intensity of the level's least-squares projection onto the 64 basis
    vectors."""
    rng = np.random.Generator(np.random.PCG64(5))
    i1 = rng.exponential(1e-8, (4, 1024))
    im = rng.exponential(1e-9, (4, 1024)) * (rng.random((4, 1024)) < 0.3)
    c = SO.level_coefficients(im)
    prof = SO.profile_from_coefficients(i1, c)
    C = SO.dct_basis(1024)
    proj = SO.level_db(im) @ C.T @ C
    np.testing.assert_allclose(prof, 10 * np.log10(i1 + SO.I_FLOOR * 10 ** (proj / 10)), atol=1e-10)


def test_level_closed_forms():
    """Level of a constant later-bounce intensity c: 10 log10(1 + c / floor)
    in every bin, so only coefficient 0 is nonzero (sqrt(n) times it); with
    the full-resolution (untruncated) level the profile is exactly the
    multi-bounce truth 10 log10(I1 + Im + floor)."""
    n = 256
    c = 3.0e-9
    im = np.full((1, n), c)
    lv = SO.level_db(im)
    np.testing.assert_allclose(lv, 10 * np.log10(1 + c / SO.I_FLOOR), rtol=1e-14)
    coef = SO.level_coefficients(im)
    np.testing.assert_allclose(coef[0, 0], np.sqrt(n) * 10 * np.log10(1 + c / SO.I_FLOOR), rtol=1e-12)
    assert np.abs(coef[0, 1:]).max() < 1e-9
    rng = np.random.Generator(np.random.PCG64(8))
    i1 = rng.exponential(1e-8, (3, 64)) * (rng.random((3, 64)) < 0.5)
    im = rng.exponential(1e-9, (3, 64)) * (rng.random((3, 64)) < 0.5)
    C = SO.dct_basis(64, 64)
    full = SO.level_db(im) @ C.T
    prof = 10 * np.log10(i1 + SO.I_FLOOR * 10 ** ((full @ C) / 10))
    np.testing.assert_allclose(prof, 10 * np.log10(i1 + im + SO.I_FLOOR), atol=1e-9)


def test_zero_later_bounce_gives_single_bounce_profile():
    i1 = np.full((2, 1024), 1e-8)
    c = SO.level_coefficients(np.zeros_like(i1))
    assert np.abs(c).max() < 1e-12
    err, n = SO.beam_errors(i1, np.zeros_like(i1), SO.profile_from_coefficients(i1, c))
    assert np.all(err < 1e-10) and np.all(n == 1024)


def test_full_profile_definitions():
    """Full-resolution profile: zero coefficients give the raw single-bounce
    profile; coefficients of a constant level c from bin 0 add the intensity
    floor (10^(c/10) - 1) to every bin from the first-hit bin on."""
    rng = np.random.Generator(np.random.PCG64(10))
    n = 128
    i1 = rng.exponential(1e-8, (3, n)) * (rng.random((3, n)) < 0.4)
    r1 = np.array([0, 17, 100])
    z = SO.full_profile(i1, np.zeros((3, 64)), r1)
    np.testing.assert_allclose(z, 10 * np.log10(i1 + SO.I_FLOOR), atol=1e-12)
    c = 6.0
    coef = np.zeros((3, 64))
    coef[:, 0] = c * np.sqrt(n)          # a constant level c over all n bins
    p = SO.full_profile(i1, coef, r1)
    for k in range(3):
        want = i1[k] + SO.I_FLOOR
        want[r1[k]:] += SO.I_FLOOR * (10 ** (c / 10) - 1)
        np.testing.assert_allclose(p[k], 10 * np.log10(want), atol=1e-9)


def test_weighted_loss_is_profile_squared_error():
    """With w_j = sigma_j^2 / mean(sigma^2) the loss on standardised
    coefficients is the mean squared error of the de-standardised
    coefficients over mean(sigma^2), i.e. (Parseval) the profile's."""
    rng = np.random.Generator(np.random.PCG64(9))
    sg = rng.uniform(0.2, 3.0, 64)
    mu = rng.normal(0, 1, 64)
    y, t = rng.normal(size=(10, 64)), rng.normal(size=(10, 64))
    w = sg ** 2 / np.mean(sg ** 2)
    loss, _ = SO.mse(y, t, w)
    raw = ((y * sg + mu) - (t * sg + mu)) @ SO.dct_basis(256, 64)
    np.testing.assert_allclose(loss, (raw ** 2).sum() / (10 * 64) / np.mean(sg ** 2), rtol=1e-12)


def test_smoothing_and_alignment_definitions():
    rng = np.random.Generator(np.random.PCG64(6))
    a = rng.random((3, 100))
    s = SO.smooth_range(a, 8)
    # interior: plain window mean; total mass preserved away from the edges
    np.testing.assert_allclose(s[:, 50], a[:, 46:54].mean(axis=1))
    np.testing.assert_allclose(s[:, 0], a[:, 0:4].sum(axis=1) / 8)
    # alignment: a level confined after r1 maps back exactly through the full basis
    i1 = np.zeros((2, 256))
    im = np.zeros((2, 256))
    i1[:, 100:120] = 1e-8
    im[:, 130:150] = 1e-8
    r1 = np.array([100, 90])
    c = SO.aligned_level_coefficients(im, r1)
    assert c.shape == (2, 64)
    prof = SO.aligned_profile(i1, c, r1)
    # the truncated reconstruction is the projection of the aligned level
    lv = SO.level_db(SO.smooth_range(im))
    C = SO.dct_basis(256)
    for k in range(2):
        al = np.zeros(256)
        al[:256 - r1[k]] = lv[k, r1[k]:]
        proj = al @ C.T @ C
        back = np.zeros(256)
        back[r1[k]:] = proj[:256 - r1[k]]
        want = 10 * np.log10(SO.smooth_range(i1)[k] + SO.I_FLOOR * 10 ** (back / 10))
        np.testing.assert_allclose(prof[k], want, atol=1e-9)


def test_first_hit_bin():
    g = np.zeros((3, 8), np.float32)
    g[0, 0], g[0, 6] = 10.0 / 15.0, 1.0
    g[1, 0], g[1, 6] = 10.0 / 15.0, 0.0          # no hits
    g[2, 0], g[2, 6] = 0.01, 0.5                 # before r_min
    b = SO.first_hit_bin(g, 0.3, 15.0, 1024)
    assert b[0] == int(np.floor((np.float32(10.0 / 15.0) * np.float32(15.0) - np.float32(0.3))
                                / np.float32(14.7 / 1024)))
    assert b[1] == 0 and b[2] == 0
