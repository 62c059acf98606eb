"""ctypes front end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg. The product package never imports it, and it
imports nothing from the product package except the seeded input generators.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Beam options (sensor flags, see oracle.c)
BEAM_PATTERN, RX_BEAMS, DIFFUSE_BOUNCE, RETRO_CHAIN = 1, 2, 4, 8

# Ambiguity flag bits (see oracle.c)
F_GRAZE, F_EDGE, F_TIE, F_LIMIT, F_SELF, F_BIN, F_FOV, F_OCCLUDER, F_STOP, F_DEPART, F_CAUSTIC = \
    (1 << i for i in range(11))
FLAG_NAMES = ("graze", "edge", "tie", "limit", "self", "bin", "fov", "occluder", "stop", "depart", "caustic")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: FP64, no fused multiply-add contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("hfov", C.c_double), ("vfov", C.c_double),
                ("n_h", C.c_int32), ("n_v", C.c_int32), ("n_r", C.c_int32),
                ("grid_mode", C.c_int32), ("jitter", C.c_int32), ("n_bins", C.c_int32),
                ("r_min", C.c_double), ("r_max", C.c_double),
                ("f0", C.c_double), ("c0", C.c_double), ("g", C.c_double),
                ("alpha_db", C.c_double),
                ("max_bounces", C.c_int32), ("pad0", C.c_int32),
                ("k_d", C.c_double), ("k_s", C.c_double), ("phong_n", C.c_double),
                ("seed", C.c_uint64), ("ping", C.c_uint32), ("flags", C.c_uint32),
                ("n_knots", C.c_int32), ("pad2", C.c_int32),
                ("knot_z", C.c_double * 8), ("knot_c", C.c_double * 8)]


class PoseS(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("rot", C.c_double * 9)]


class Tol(C.Structure):
    _fields_ = [("graze", C.c_double), ("edge_abs", C.c_double), ("edge_rel", C.c_double),
                ("tie_rel", C.c_double), ("tie_abs", C.c_double), ("bin_frac", C.c_double),
                ("fov", C.c_double), ("lim_rel", C.c_double),
                ("self_lo", C.c_double), ("self_hi", C.c_double), ("caustic", C.c_double)]


class Cfar(C.Structure):
    _fields_ = [("train", C.c_int32), ("guard", C.c_int32), ("max_per_beam", C.c_int32),
                ("pad", C.c_int32), ("pfa", C.c_double), ("noise_floor", C.c_double)]


def default_tol(**kw) -> Tol:
    """Flag margins: grazing below cos 1e-3, hits within 2e-5 m + 2e-6 s of an
    edge, second candidates within 1e-5 relative + 1e-6 m, range positions within
    1e-6 of a bin edge, arrival directions within 1e-9 rad of the FOV edge,
    bounds within 1e-7 relative, hit distances in [5e-5, 2e-4] m, and in a
    layered profile two eigenrays turning within 1/64 of the turning-depth
    window of each other."""
    t = dict(graze=1e-3, edge_abs=2e-5, edge_rel=2e-6, tie_rel=1e-5, tie_abs=1e-6,
             bin_frac=1e-6, fov=1e-9, lim_rel=1e-7, self_lo=5e-5, self_hi=2e-4, caustic=1.0 / 64)
    t.update(kw)
    return Tol(**t)


def zero_tol() -> Tol:
    return Tol(graze=0, edge_abs=0, edge_rel=0, tie_rel=0, tie_abs=0, bin_frac=0, fov=0,
               lim_rel=0, self_lo=1e-4, self_hi=1e-4, caustic=0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P = C.POINTER
        L.orc_scene_new.restype = C.c_void_p
        L.orc_scene_new.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_scene_free.argtypes = [C.c_void_p]
        L.orc_scene_build_grid.argtypes = [C.c_void_p, C.c_double]
        L.orc_scene_grid_info.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_grid_counts.argtypes = [C.c_double] * 7 + [C.c_void_p]
        L.orc_splitmix64_nth.restype = C.c_uint64
        L.orc_splitmix64_nth.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_jitter.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p]
        L.orc_ray.argtypes = [P(Params), P(PoseS), C.c_int32, C.c_int32, C.c_void_p]
        L.orc_connection.argtypes = [P(Params), C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_path_eval.argtypes = [P(Params), C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
        L.orc_eigenray.argtypes = [P(Params), P(Tol), C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
        L.orc_trace_beams.restype = C.c_int
        L.orc_trace_beams.argtypes = [C.c_void_p, P(Params), P(PoseS), P(Tol), C.c_void_p, C.c_int64] + \
            [C.c_void_p] * 12 + [C.c_int]
        L.orc_draw_continuation.argtypes = [P(Params), C.c_uint64, C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                            C.c_double, C.c_void_p]
        L.orc_trace_one.restype = C.c_int
        L.orc_trace_one.argtypes = [C.c_void_p, P(Params), P(PoseS), P(Tol), C.c_void_p, C.c_void_p] + [C.c_void_p] * 7
        L.orc_detect.restype = C.c_int
        L.orc_detect.argtypes = [C.c_void_p, P(Params), P(PoseS), P(Cfar), C.c_void_p, C.c_int64] + \
            [C.c_void_p] * 5 + [C.c_double, C.c_double]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def params_of(cfg, ping: int = 0) -> Params:
    """Oracle parameters from a ``scenes.SensorConfig`` (``cfg.ssp``: knots
    (z, c) of a piecewise-linear sound speed, or empty)."""
    p = _params(cfg, ping)
    knots = list(getattr(cfg, "ssp", ()) or ())
    p.n_knots = len(knots)
    for i, (z, c) in enumerate(knots[:8]):
        p.knot_z[i] = z
        p.knot_c[i] = c
    return p


def _params(cfg, ping: int = 0) -> Params:
    return Params(hfov=cfg.hfov, vfov=cfg.vfov, n_h=cfg.n_h, n_v=cfg.n_v, n_r=cfg.rays_per_beam,
                  grid_mode=cfg.grid_mode, jitter=cfg.jitter, n_bins=cfg.n_range,
                  r_min=cfg.r_min, r_max=cfg.r_max, f0=cfg.freq_hz, c0=cfg.c0, g=cfg.c_grad,
                  alpha_db=cfg.abs_db_per_m, max_bounces=cfg.max_bounces, pad0=0,
                  k_d=cfg.k_d, k_s=cfg.k_s, phong_n=cfg.phong_n, seed=cfg.seed, ping=ping,
                  flags=int(cfg.flags) & (BEAM_PATTERN | RX_BEAMS | DIFFUSE_BOUNCE | RETRO_CHAIN))


def pose_of(pose) -> PoseS:
    q = PoseS()
    for i in range(3):
        q.pos[i] = pose.position[i]
    for i in range(9):
        q.rot[i] = pose.rot[i]
    return q


GRID_MIN_TRIANGLES = 20000


class Scene:
    """The oracle's copy of a mesh. ``grid``: bin the triangles in a uniform
    grid used as an exact candidate filter (every query visits, in index
    order, every triangle that could change its result or flags; the
    arithmetic per triangle is the brute-force one). Default: on for meshes
    of at least GRID_MIN_TRIANGLES triangles."""

    def __init__(self, mesh, grid=None, cells_per_triangle: float = 0.5):
        self._keep = (np.ascontiguousarray(mesh.vertices, np.float32),
                      np.ascontiguousarray(mesh.indices, np.int32),
                      np.ascontiguousarray(mesh.reflectivity, np.float32),
                      np.ascontiguousarray(mesh.phase, np.float32),
                      np.ascontiguousarray(mesh.material, np.uint8))
        v, i, r, p, m = self._keep
        self.h = lib().orc_scene_new(_ptr(v), v.shape[0], _ptr(i), i.shape[0], _ptr(r), _ptr(p), _ptr(m))
        self.n_triangles = i.shape[0]
        if grid is None:
            grid = self.n_triangles >= GRID_MIN_TRIANGLES
        if grid:
            lib().orc_scene_build_grid(self.h, float(cells_per_triangle))

    def grid_info(self) -> dict:
        out = np.zeros(3)
        lib().orc_scene_grid_info(self.h, _ptr(out))
        return dict(cells=int(out[0]), entries=int(out[1]), cell=float(out[2]))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_scene_free(self.h)
            self.h = None


def grid_counts(hfov, vfov, dth_h, dth_v, r_min, r_max, dr):
    out = np.zeros(6, np.int32)
    lib().orc_grid_counts(hfov, vfov, dth_h, dth_v, r_min, r_max, dr, _ptr(out))
    return dict(zip(("n_range", "n_h", "n_v", "n_l", "n_r", "n_e"), (int(x) for x in out)))


def splitmix64_nth(seed: int, n: int) -> int:
    return int(lib().orc_splitmix64_nth(seed, n))


def jitter(seed, ping, beam, ray):
    out = np.zeros(2)
    lib().orc_jitter(seed, ping, beam, ray, _ptr(out))
    return out


def ray(cfg, pose, beam, j):
    out = np.zeros(6)
    lib().orc_ray(C.byref(params_of(cfg, pose.ping)), C.byref(pose_of(pose)), beam, j, _ptr(out))
    return out[:3], out[3:]


def connection(cfg, p, s):
    out = np.zeros(8)
    lib().orc_connection(C.byref(params_of(cfg)), _ptr(np.asarray(p, np.float64)),
                         _ptr(np.asarray(s, np.float64)), _ptr(out))
    return dict(L=out[0], T=out[1], w_out=out[2:5], arrive=out[5:8])


def eigenray(cfg, p, s, H=None, tol=None):
    """The layered profile's first-arriving eigenray from p to s (turning
    depths within H of the span, 2 r_max by default): ok, family (0 direct,
    1 turning above, 2 turning below), number of roots, invariant xi, turning
    depth, L, T, departure and arrival directions, flags."""
    out = np.zeros(14)
    H = 2.0 * cfg.r_max if H is None else H
    lib().orc_eigenray(C.byref(params_of(cfg)), C.byref(tol or default_tol()), _ptr(np.asarray(p, np.float64)),
                       _ptr(np.asarray(s, np.float64)), float(H), _ptr(out))
    return dict(ok=bool(out[0]), fam=int(out[1]), n_roots=int(out[2]), xi=out[3], zt=out[4], L=out[5], T=out[6],
                w_out=out[7:10], arrive=out[10:13], flags=int(out[13]))


def path_eval(cfg, o, d, s):
    out = np.zeros(7)
    lib().orc_path_eval(C.byref(params_of(cfg)), _ptr(np.asarray(o, np.float64)),
                        _ptr(np.asarray(d, np.float64)), float(s), _ptr(out))
    return out[:3], out[3:6], out[6]


def trace_beams(scene: Scene, cfg, pose, beams, tol=None, threads: int = 0, want_all=True,
                want_incoh=False, want_gbuf=False):
    """All rays of the listed beams. Returns a dict of numpy arrays:
    col [nb, n_bins] complex128 (flagged rays excluded), col_all (every ray),
    incoh [nb, 2, n_bins], gbuf [nb, 8], tri/bin/vis [nb*n_r, K], amp [nb*n_r, K]
    complex128, flags [nb*n_r]."""
    beams = np.ascontiguousarray(beams, np.int32)
    nb = beams.shape[0]
    P = params_of(cfg, pose.ping)
    K, NB, NR = cfg.max_bounces, cfg.n_range, cfg.rays_per_beam
    col = np.zeros((nb, NB, 2))
    col_all = np.zeros((nb, NB, 2)) if want_all else None
    incoh = np.zeros((nb, 2, NB)) if want_incoh else None
    gbuf = np.zeros((nb, 8)) if want_gbuf else None
    tri = np.zeros((nb * NR, K), np.int32)
    bin_ = np.zeros((nb * NR, K), np.int32)
    vis = np.zeros((nb * NR, K), np.int32)
    amp = np.zeros((nb * NR, K, 2))
    flags = np.zeros(nb * NR, np.uint32)
    rxb = np.zeros((nb * NR, K), np.int32)
    rbin = np.zeros((nb * NR, K), np.int32)
    ramp = np.zeros((nb * NR, K, 2))
    tol = tol if tol is not None else default_tol()
    rc = lib().orc_trace_beams(scene.h, C.byref(P), C.byref(pose_of(pose)), C.byref(tol), _ptr(beams), nb,
                               _ptr(col), _ptr(col_all), _ptr(incoh), _ptr(gbuf), _ptr(tri), _ptr(bin_),
                               _ptr(vis), _ptr(amp), _ptr(flags), _ptr(rxb), _ptr(rbin), _ptr(ramp), int(threads))
    if rc != 0:
        raise ValueError(f"oracle rejected the parameters ({rc})")
    out = dict(col=col[..., 0] + 1j * col[..., 1], tri=tri, bin=bin_, vis=vis,
               amp=amp[..., 0] + 1j * amp[..., 1], flags=flags, rxb=rxb,
               rbin=rbin, ramp=ramp[..., 0] + 1j * ramp[..., 1])
    if want_all:
        out["col_all"] = col_all[..., 0] + 1j * col_all[..., 1]
    if want_incoh:
        out["incoh"] = incoh
    if want_gbuf:
        out["gbuf"] = gbuf
    return out


def draw_continuation(cfg, ping, ray, k, rh, np_, kd, ks):
    out = np.zeros(5)
    lib().orc_draw_continuation(C.byref(params_of(cfg, ping)), int(ray), int(k),
                                _ptr(np.asarray(rh, np.float64)), _ptr(np.asarray(np_, np.float64)), float(kd),
                                float(ks), _ptr(out))
    return out[:3], float(out[3]), bool(out[4])


def trace_one(scene: Scene, cfg, pose, o, d, tol=None):
    K = cfg.max_bounces
    tri = np.zeros(K, np.int32)
    bin_ = np.zeros(K, np.int32)
    vis = np.zeros(K, np.int32)
    amp = np.zeros((K, 2))
    fl = np.zeros(1, np.uint32)
    rbin = np.zeros(K, np.int32)
    ramp = np.zeros((K, 2))
    tol = tol if tol is not None else default_tol()
    lib().orc_trace_one(scene.h, C.byref(params_of(cfg, pose.ping)), C.byref(pose_of(pose)), C.byref(tol),
                        _ptr(np.asarray(o, np.float64)), _ptr(np.asarray(d, np.float64)),
                        _ptr(tri), _ptr(bin_), _ptr(vis), _ptr(amp), _ptr(fl), _ptr(rbin), _ptr(ramp))
    return dict(tri=tri, bin=bin_, vis=vis, amp=amp[:, 0] + 1j * amp[:, 1], flags=int(fl[0]),
                rbin=rbin, ramp=ramp[:, 0] + 1j * ramp[:, 1])


def detect(volume, cfg, pose, beams, train=16, guard=4, max_per_beam=4, pfa=1e-4, noise_floor=1e-11,
           rel_thr=1e-4, rel_peak=1e-6):
    """CA-CFAR + peak detection of the listed beams of a complex64 volume
    [n_beams_total, n_bins]. Returns dict(bin [nb, M], pts [nb, M, 4], count [nb],
    flag_bins [nb, n_bins], beam_flag [nb])."""
    vol = np.ascontiguousarray(np.asarray(volume).astype(np.complex64)).view(np.float32)
    beams = np.ascontiguousarray(beams, np.int32)
    nb, M, NB = beams.shape[0], max_per_beam, cfg.n_range
    out_bin = np.zeros((nb, M), np.int32)
    pts = np.zeros((nb, M, 4))
    cnt = np.zeros(nb, np.int32)
    fb = np.zeros((nb, NB), np.uint8)
    bf = np.zeros(nb, np.int32)
    cf = Cfar(train=train, guard=guard, max_per_beam=M, pad=0, pfa=pfa, noise_floor=noise_floor)
    lib().orc_detect(_ptr(vol), C.byref(params_of(cfg, pose.ping)), C.byref(pose_of(pose)), C.byref(cf),
                     _ptr(beams), nb, _ptr(out_bin), _ptr(pts), _ptr(cnt), _ptr(fb), _ptr(bf), rel_thr, rel_peak)
    return dict(bin=out_bin, pts=pts, count=cnt, flag_bins=fb, beam_flag=bf)
