"""The C-ABI library loads, exports every declared symbol and validates its
arguments on the host (no GPU needed: nothing here launches a kernel)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_2606_06130_amd import scenes as S
from paper_2606_06130_amd import sonar

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sonar.h")).read()
    return sorted(set(re.findall(r"\b(sonar_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sonar.LIB_PATH):
        pytest.skip("libsonar.so not built")
    return sonar.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert sorted(sonar.EXPORTS) == names


def test_status_strings(L):
    for st in (0, 1, -1, -2, -3, -4, -5):
        assert L.sonar_status_string(st)
    assert L.sonar_status_string(99) == b"unknown status"


def test_params_from_resolution_eq1_3(L):
    p = sonar.params_from_resolution(math.radians(90), math.radians(40), math.radians(1.40625), math.radians(1.25),
                                     0.3, 15.0, 14.7 / 256)
    assert (p.n_h, p.n_v, p.n_range) == (64, 32, 256)
    with pytest.raises(sonar.SonarError):
        sonar.params_from_resolution(math.radians(90), math.radians(40), 0.0, 1.0, 0.3, 15.0, 0.1)


def test_ping_rejects_null_scene(L):
    p = sonar.params_of(S.sensor_seabed_boxes())
    q = sonar.pose_of(S.pose_seabed_boxes())
    st = L.sonar_ping(None, C.byref(p), C.byref(q), C.c_void_p(16), None, None, None, None, None)
    assert st == sonar.SONAR_E_INVALID
    assert b"scene" in L.sonar_last_error()


@pytest.mark.parametrize("field,value", [("n_h", 0), ("rays_per_beam", 3), ("rays_per_beam", 128),
                                         ("n_range", 0), ("n_range", 5000), ("max_bounces", 0),
                                         ("max_bounces", 5), ("r_max", 0.1), ("hfov", 0.0), ("c0", -1.0),
                                         ("grid_mode", 2), ("k_s", -0.5)])
def test_detect_validates_params_before_launch(L, field, value):
    cfg = S.sensor_seabed_boxes()
    p = sonar.params_of(cfg)
    setattr(p, field, value)
    q = sonar.pose_of(S.pose_seabed_boxes())
    c = sonar.sonar_cfar(train=16, guard=4, max_per_beam=4, pad=0, pfa=1e-4, noise_floor=1e-11)
    st = L.sonar_detect(C.c_void_p(16), C.byref(p), C.byref(q), C.byref(c), C.c_void_p(16), 10, C.c_void_p(16),
                        C.c_void_p(16), 1 << 30, None)
    assert st == sonar.SONAR_E_INVALID
    assert L.sonar_detect_workspace_size(C.byref(p)) == 0


def test_detect_validates_cfar_and_pose(L):
    cfg = S.sensor_seabed_boxes()
    p = sonar.params_of(cfg)
    q = sonar.pose_of(S.pose_seabed_boxes())
    ws = L.sonar_detect_workspace_size(C.byref(p))
    assert ws >= cfg.n_beams * 4 * 2
    for kw in (dict(max_per_beam=0), dict(max_per_beam=17), dict(pfa=0.0), dict(pfa=1.0), dict(train=0)):
        args = dict(train=16, guard=4, max_per_beam=4, pad=0, pfa=1e-4, noise_floor=1e-11)
        args.update(kw)
        c = sonar.sonar_cfar(**args)
        st = L.sonar_detect(C.c_void_p(16), C.byref(p), C.byref(q), C.byref(c), C.c_void_p(16), 10, C.c_void_p(16),
                            C.c_void_p(16), ws, None)
        assert st == sonar.SONAR_E_INVALID, kw
    c = sonar.sonar_cfar(train=16, guard=4, max_per_beam=4, pad=0, pfa=1e-4, noise_floor=1e-11)
    st = L.sonar_detect(C.c_void_p(16), C.byref(p), C.byref(q), C.byref(c), C.c_void_p(16), 10, C.c_void_p(16),
                        C.c_void_p(16), ws - 1, None)
    assert st == sonar.SONAR_E_INVALID and b"workspace" in L.sonar_last_error()
    bad = sonar.pose_of(S.pose_seabed_boxes())
    bad.rot[0] = 2.0
    st = L.sonar_detect(C.c_void_p(16), C.byref(p), C.byref(bad), C.byref(c), C.c_void_p(16), 10, C.c_void_p(16),
                        C.c_void_p(16), ws, None)
    assert st == sonar.SONAR_E_INVALID and b"orthonormal" in L.sonar_last_error()


def test_build_rejects_null_mesh(L):
    out = C.c_void_p()
    assert L.sonar_build_scene(None, None, C.byref(out)) == sonar.SONAR_E_INVALID
    m = sonar.sonar_mesh()
    assert L.sonar_build_scene(C.byref(m), None, C.byref(out)) == sonar.SONAR_E_INVALID
    assert out.value is None


@pytest.mark.parametrize("B,tau,dt,window", [(40e3, 300e-6, 19.14e-6, 0), (40e3, 300e-6, 19.14e-6, 1),
                                             (0.0, 1e-4, 1e-5, 0), (1e5, 5e-6, 1e-5, 1), (0.4, 64.0, 1.0, 0)])
def test_lfm_pulse_matches_oracle(L, B, tau, dt, window):
    from oracle import pulse as OP
    got = sonar.lfm_pulse(B, tau, dt, window)
    want = OP.lfm_pulse(B, tau, dt, window)
    assert got.dtype == np.complex64 and got.shape == want.shape
    assert np.abs(got - want).max() <= 2e-7          # FP32 rounding of unit-magnitude taps


def test_lfm_pulse_rejects(L):
    for args in [(-1.0, 1e-4, 1e-5, 0), (1e3, 0.0, 1e-5, 0), (1e3, 1e-4, 0.0, 0), (1e3, 1e-4, 1e-5, 2),
                 (1e3, 65e-5, 1e-5, 0)]:
        with pytest.raises(sonar.SonarError) as e:
            sonar.lfm_pulse(*args)
        assert e.value.status == sonar.SONAR_E_INVALID
    taps = (C.c_float * 8)()
    n = C.c_int32()
    assert L.sonar_lfm_pulse(1e3, 10e-5, 1e-5, 0, taps, 4, C.byref(n)) == sonar.SONAR_E_INVALID   # 10 taps > 4


def test_pulse_compress_validates_before_launch(L):
    p = (C.c_float * 4)(1.0, 0.0, 0.5, 0.5)
    vol, out1, out2 = C.c_void_p(0x100000), C.c_void_p(0x900000), C.c_void_p(0x1100000)
    E = sonar.SONAR_E_INVALID
    assert L.sonar_pulse_compress(None, 4, 16, p, 2, out1, out2, None) == E
    assert L.sonar_pulse_compress(vol, 4, 16, None, 2, out1, out2, None) == E
    assert L.sonar_pulse_compress(vol, 4, 16, p, 2, None, None, None) == E          # no output
    assert L.sonar_pulse_compress(vol, -1, 16, p, 2, out1, None, None) == E
    assert L.sonar_pulse_compress(vol, 4, 0, p, 2, out1, None, None) == E
    assert L.sonar_pulse_compress(vol, 4, 2049, p, 2, out1, None, None) == E
    assert L.sonar_pulse_compress(vol, 4, 16, p, 0, out1, None, None) == E
    assert L.sonar_pulse_compress(vol, 4, 16, p, 65, out1, None, None) == E
    assert L.sonar_pulse_compress(vol, 4, 16, p, 2, C.c_void_p(0x100000 + 8), None, None) == E   # overlaps input
    assert b"overlap" in L.sonar_last_error()
    assert L.sonar_pulse_compress(vol, 4, 16, p, 2, out1, C.c_void_p(0x900000 + 64), None) == E  # outputs overlap
    assert L.sonar_pulse_compress(vol, 0, 16, p, 2, out1, None, None) == 0                       # nothing to do


def test_rx_workspace_size(L):
    cfg = S.sensor_seabed_boxes().replace(n_h=16, n_v=8, rays_per_beam=4, max_bounces=3)
    p = sonar.params_of(cfg)
    assert L.sonar_rx_workspace_size(C.byref(p)) == 256                      # no receive binning
    p = sonar.params_of(cfg.replace(flags=sonar.FLAG_RX_BEAMS))
    assert L.sonar_rx_workspace_size(C.byref(p)) == 256 + 16 * 16 * 8 * 4 * 2
    p = sonar.params_of(cfg.replace(flags=sonar.FLAG_RX_BEAMS, max_bounces=1))
    assert L.sonar_rx_workspace_size(C.byref(p)) == 256
    p = sonar.params_of(cfg.replace(flags=sonar.FLAG_RETRO_CHAIN))
    assert L.sonar_rx_workspace_size(C.byref(p)) == 256                      # retro-chain returns need no list
    p = sonar.params_of(cfg.replace(flags=16))
    assert L.sonar_rx_workspace_size(C.byref(p)) == 0                        # unknown flag
    p = sonar.params_of(cfg.replace(flags=sonar.FLAG_BEAM_PATTERN, grid_mode=1, rays_per_beam=1))
    assert L.sonar_rx_workspace_size(C.byref(p)) == 0                        # cell beams only
    # the detection workspace grows by the list when a ping_detect needs it
    a = L.sonar_detect_workspace_size(C.byref(sonar.params_of(cfg)))
    b = L.sonar_detect_workspace_size(C.byref(sonar.params_of(cfg.replace(flags=sonar.FLAG_RX_BEAMS))))
    assert b >= a + 256 + 16 * 16 * 8 * 4 * 2


def test_batch_rx_workspace_size(L):
    """The batch's list workspace: each receive-binning ping's area (as for
    one ping) rounded up to 256 bytes, in ping order; 0 without such pings
    or with an invalid parameter set."""
    base = S.sensor_seabed_boxes().replace(max_bounces=2, flags=sonar.FLAG_RX_BEAMS)
    cfgs = [base.replace(n_h=9, n_v=5, rays_per_beam=1),            # 256 + 16 * 45 = 976 -> 1,024
            base.replace(n_h=16, n_v=8, rays_per_beam=4, flags=0),  # no list
            base.replace(n_h=16, n_v=8, rays_per_beam=4)]           # 256 + 16 * 512 = 8,448 -> 8,448
    P = (sonar.sonar_params * 3)(*[sonar.params_of(c) for c in cfgs])
    assert L.sonar_batch_rx_workspace_size(3, P) == 1024 + 8448
    for i, c in enumerate(cfgs):
        one = L.sonar_rx_workspace_size(C.byref(P[i]))
        assert L.sonar_batch_rx_workspace_size(1, C.byref(P[i])) == (((one + 255) // 256) * 256 if c.flags else 0)
    Q = (sonar.sonar_params * 2)(sonar.params_of(cfgs[1]), sonar.params_of(cfgs[1].replace(max_bounces=3)))
    assert L.sonar_batch_rx_workspace_size(2, Q) == 0
    Q[1] = sonar.params_of(cfgs[0].replace(flags=16))                  # unknown flag
    assert L.sonar_batch_rx_workspace_size(2, Q) == 0
    assert L.sonar_batch_rx_workspace_size(0, P) == 0
    assert L.sonar_batch_rx_workspace_size(2, None) == 0


def test_add_reverb_validates_before_launch(L):
    cfg = S.sensor_seabed_boxes()
    p = sonar.params_of(cfg)
    q = sonar.pose_of(S.pose_seabed_boxes())
    vol = C.c_void_p(0x100000)
    good = sonar.sonar_reverb(sv_db=-40.0, noise_power=0.0, seed=1)
    assert L.sonar_add_reverb(None, C.byref(p), C.byref(q), C.byref(good), None) == sonar.SONAR_E_INVALID
    assert L.sonar_add_reverb(vol, C.byref(p), C.byref(q), None, None) == sonar.SONAR_E_INVALID
    for bad in (sonar.sonar_reverb(sv_db=float("inf"), noise_power=0.0, seed=1),
                sonar.sonar_reverb(sv_db=-40.0, noise_power=-1.0, seed=1),
                sonar.sonar_reverb(sv_db=float("nan"), noise_power=0.0, seed=1)):
        assert L.sonar_add_reverb(vol, C.byref(p), C.byref(q), C.byref(bad), None) == sonar.SONAR_E_INVALID
    p1 = sonar.params_of(cfg.replace(grid_mode=1, rays_per_beam=1))
    assert L.sonar_add_reverb(vol, C.byref(p1), C.byref(q), C.byref(good), None) == sonar.SONAR_E_UNSUPPORTED


@pytest.mark.parametrize("g,z,knots", [(0.0, -3.0, ()), (0.05, -3.0, ()), (-0.08, 1.25, ()),
                                       (0.0, -2.0, ((-9.0, 1497.0), (-3.0, 1499.0), (1.5, 1500.3))),
                                       (0.0, -9.5, ((-9.0, 1497.0), (-3.0, 1499.0), (1.5, 1500.3))),
                                       (0.0, 2.5, ((-9.0, 1497.0), (-3.0, 1499.0), (1.5, 1500.3)))])
def test_pulse_dt_is_two_bin_widths_over_sensor_speed(L, g, z, knots):
    """dt = 2 dr / c(z_sensor): the gradient's c0 + g z, or the layered
    profile interpolated in the layer holding z (end layers extended)."""
    cfg = S.sensor_harbor().replace(c_grad=g, ssp=knots)
    pose = S.pose((0.0, 0.0, z))
    if knots:
        zs, cs = np.array([k[0] for k in knots]), np.array([k[1] for k in knots])
        i = int(np.clip(np.searchsorted(zs, z, side="right") - 1, 0, len(zs) - 2))
        c = cs[i] + (cs[i + 1] - cs[i]) / (zs[i + 1] - zs[i]) * (z - zs[i])
    else:
        c = cfg.c0 + g * z
    dr = (cfg.r_max - cfg.r_min) / cfg.n_range
    assert sonar.pulse_dt(cfg, pose) == pytest.approx(2 * dr / c, rel=1e-14)


def test_pulse_dt_rejects(L):
    p = sonar.params_of(S.sensor_harbor())
    q = sonar.pose_of(S.pose_harbor())
    assert L.sonar_pulse_dt(C.byref(p), C.byref(q), None, None) == sonar.SONAR_E_INVALID
    bad = sonar.ssp_of(((0.0, 1500.0), (-1.0, 1490.0)))
    dt = C.c_double()
    assert L.sonar_pulse_dt(C.byref(p), C.byref(q), C.byref(bad), C.byref(dt)) == sonar.SONAR_E_INVALID


def test_surrogate_geometry_block(L):
    """The surrogate's per-ping geometry block: sensor position, rotation
    row-major, fields of view, two zeros; the oracle's block of the same pose
    equals it; the LiDAR grid and bad fields of view are rejected."""
    from oracle import surrogate as SO
    cfg = S.sensor_harbor_multipath()
    poses = [S.pose((1.5, -2.0, -3.25), yaw=0.3, pitch_down=0.4), S.pose((0.0, 4.0, -1.0), yaw=-1.1)]
    blk = sonar.surrogate_geometry(cfg, poses)
    assert blk.shape == (2, 16) and blk.dtype == np.float32
    for i, p in enumerate(poses):
        want = SO.geometry_block(p.position, p.rot, cfg.hfov, cfg.vfov).astype(np.float32)
        np.testing.assert_array_equal(blk[i], want)
    with pytest.raises(sonar.SonarError):
        sonar.surrogate_geometry(cfg.replace(grid_mode=1), poses[:1])
    with pytest.raises(sonar.SonarError):
        sonar.surrogate_geometry(cfg.replace(vfov=0.0), poses[:1])
