"""Thin Python binding of ``libsonar.so`` (ctypes).

Argument marshalling only: every step of a ping runs in the library's HIP
kernels. PyTorch provides device memory (tensors) and streams. There is no
fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsonar.so")

SONAR_OK = 0
SONAR_W_TRUNCATED = 1
SONAR_E_INVALID = -1
SONAR_E_NOMEM = -2
SONAR_E_DEVICE = -3
SONAR_E_STACK = -4
SONAR_E_UNSUPPORTED = -5
FLAG_BEAM_PATTERN = 1
FLAG_RX_BEAMS = 2
FLAG_DIFFUSE_BOUNCE = 4
FLAG_RETRO_CHAIN = 8

# Every symbol include/sonar.h declares.
EXPORTS = ("sonar_build_scene", "sonar_free_scene", "sonar_get_scene_info", "sonar_ping",
           "sonar_detect_workspace_size", "sonar_detect", "sonar_ping_detect", "sonar_device_status",
           "sonar_status_string", "sonar_last_error", "sonar_params_from_resolution",
           "sonar_batch_desc_bytes", "sonar_batch_workspace_size", "sonar_batch_prepare", "sonar_ping_batch",
           "sonar_batch_stamps", "sonar_batch_graph_create", "sonar_graph_launch", "sonar_graph_free",
           "sonar_batch_autotune", "sonar_batch_emit_desc_bytes", "sonar_batch_detect_workspace_size",
           "sonar_batch_prepare_detect", "sonar_surrogate_param_count", "sonar_surrogate_create",
           "sonar_surrogate_free", "sonar_surrogate_set_state", "sonar_surrogate_get_state",
           "sonar_surrogate_set_norm", "sonar_surrogate_geometry", "sonar_surrogate_forward",
           "sonar_surrogate_train_step",
           "sonar_surrogate_gradient", "sonar_surrogate_target", "sonar_surrogate_moments",
           "sonar_surrogate_set_loss_weights",
           "sonar_surrogate_profile", "sonar_lfm_pulse", "sonar_pulse_compress",
           "sonar_rx_workspace_size", "sonar_ping_rx", "sonar_add_reverb",
           "sonar_ping_ssp", "sonar_ping_ssp_rx", "sonar_batch_prepare_ssp", "sonar_batch_rx_workspace_size",
           "sonar_batch_prepare_rx", "sonar_batch_set_outputs", "sonar_ping_detect_noalloc",
           "sonar_workspace_size", "sonar_ping_ws", "sonar_pulse_dt")


class SonarError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class sonar_mesh(C.Structure):
    _fields_ = [("vertices", C.c_void_p), ("indices", C.c_void_p), ("reflectivity", C.c_void_p),
                ("phase", C.c_void_p), ("material", C.c_void_p), ("n_vertices", C.c_int64),
                ("n_triangles", C.c_int64), ("on_device", C.c_int32), ("leaf_size", C.c_int32)]


class sonar_pose(C.Structure):
    _fields_ = [("position", C.c_double * 3), ("rot", C.c_double * 9), ("ping", C.c_uint32), ("pad", C.c_uint32)]


class sonar_params(C.Structure):
    _fields_ = [("hfov", C.c_double), ("vfov", C.c_double),
                ("n_h", C.c_int32), ("n_v", C.c_int32), ("rays_per_beam", C.c_int32), ("grid_mode", C.c_int32),
                ("jitter", C.c_int32), ("n_range", C.c_int32),
                ("r_min", C.c_double), ("r_max", C.c_double), ("freq_hz", C.c_double), ("c0", C.c_double),
                ("c_grad", C.c_double), ("abs_db_per_m", C.c_double),
                ("max_bounces", C.c_int32), ("pad0", C.c_int32),
                ("k_d", C.c_double), ("k_s", C.c_double), ("phong_n", C.c_double),
                ("seed", C.c_uint64), ("flags", C.c_uint32), ("pad1", C.c_uint32)]


class sonar_cfar(C.Structure):
    _fields_ = [("train", C.c_int32), ("guard", C.c_int32), ("max_per_beam", C.c_int32), ("pad", C.c_int32),
                ("pfa", C.c_double), ("noise_floor", C.c_double)]


class sonar_ray_record(C.Structure):
    _fields_ = [("tri", C.c_void_p), ("bin", C.c_void_p), ("vis", C.c_void_p), ("amp", C.c_void_p),
                ("stats", C.c_void_p), ("beam", C.c_void_p), ("retro_bin", C.c_void_p),
                ("retro_amp", C.c_void_p)]


class sonar_scene_info(C.Structure):
    _fields_ = [("n_triangles", C.c_int64), ("n_nodes", C.c_int64), ("depth", C.c_int32),
                ("leaf_size", C.c_int32), ("lo", C.c_float * 3), ("hi", C.c_float * 3),
                ("node_bytes", C.c_int64), ("tri_bytes", C.c_int64)]


class sonar_ssp(C.Structure):
    _fields_ = [("n_knots", C.c_int32), ("pad", C.c_int32), ("z", C.c_double * 8), ("c", C.c_double * 8)]


def ssp_of(knots) -> sonar_ssp:
    """sonar_ssp from knots [(z, c), ...]."""
    q = sonar_ssp(n_knots=len(knots))
    for i, (z, c) in enumerate(knots[:8]):
        q.z[i] = z
        q.c[i] = c
    return q


class sonar_reverb(C.Structure):
    _fields_ = [("sv_db", C.c_double), ("noise_power", C.c_double), ("seed", C.c_uint64)]


class sonar_batch_plan(C.Structure):
    _fields_ = [("n_pings", C.c_int32), ("max_bounces", C.c_int32), ("arc", C.c_int32), ("max_bins", C.c_int32),
                ("max_beams", C.c_int32), ("retro", C.c_int32), ("rx", C.c_int32),
                ("total_tiles", C.c_int64),
                ("total_rays", C.c_int64)]


class sonar_batch_options(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int32), ("tiles_per_item", C.c_int32), ("emit_desc", C.c_void_p),
                ("waves_per_block", C.c_int32), ("pad", C.c_int32)]


POINT_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("db", "<f4"), ("beam", "<i4"), ("bin", "<i4")])

_lib = None


def lib():
    """Loads libsonar.so (built by ``paper_2606_06130_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2606_06130_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.sonar_build_scene.restype = C.c_int
        L.sonar_build_scene.argtypes = [P(sonar_mesh), C.c_void_p, P(C.c_void_p)]
        L.sonar_free_scene.restype = None
        L.sonar_free_scene.argtypes = [C.c_void_p]
        L.sonar_get_scene_info.restype = C.c_int
        L.sonar_get_scene_info.argtypes = [C.c_void_p, P(sonar_scene_info)]
        L.sonar_ping.restype = C.c_int
        L.sonar_ping.argtypes = [C.c_void_p, P(sonar_params), P(sonar_pose), C.c_void_p, C.c_void_p, C.c_void_p,
                                 P(sonar_ray_record), C.c_void_p, C.c_void_p]
        L.sonar_detect_workspace_size.restype = C.c_size_t
        L.sonar_detect_workspace_size.argtypes = [P(sonar_params)]
        L.sonar_detect.restype = C.c_int
        L.sonar_detect.argtypes = [C.c_void_p, P(sonar_params), P(sonar_pose), P(sonar_cfar), C.c_void_p, C.c_int32,
                                   C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.sonar_ping_detect.restype = C.c_int
        L.sonar_ping_detect.argtypes = [C.c_void_p, P(sonar_params), P(sonar_pose), P(sonar_cfar), C.c_void_p,
                                        C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.sonar_ping_detect_noalloc.restype = C.c_int
        L.sonar_ping_detect_noalloc.argtypes = [C.c_void_p, P(sonar_params), P(sonar_pose), P(sonar_cfar),
                                                C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.sonar_device_status.restype = C.c_int
        L.sonar_device_status.argtypes = [C.c_void_p, C.c_void_p]
        L.sonar_status_string.restype = C.c_char_p
        L.sonar_status_string.argtypes = [C.c_int]
        L.sonar_last_error.restype = C.c_char_p
        L.sonar_last_error.argtypes = []
        L.sonar_batch_desc_bytes.restype = C.c_size_t
        L.sonar_batch_desc_bytes.argtypes = []
        L.sonar_batch_workspace_size.restype = C.c_size_t
        L.sonar_batch_workspace_size.argtypes = [C.c_int32]
        L.sonar_batch_prepare.restype = C.c_int
        L.sonar_batch_prepare.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          P(sonar_batch_plan)]
        L.sonar_batch_prepare_ssp.restype = C.c_int
        L.sonar_batch_prepare_ssp.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, P(sonar_ssp), C.c_void_p,
                                              C.c_void_p, P(sonar_batch_plan)]
        L.sonar_batch_rx_workspace_size.restype = C.c_size_t
        L.sonar_batch_rx_workspace_size.argtypes = [C.c_int32, C.c_void_p]
        L.sonar_batch_prepare_rx.restype = C.c_int
        L.sonar_batch_prepare_rx.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_void_p, C.c_size_t, C.c_void_p, P(sonar_batch_plan)]
        L.sonar_batch_set_outputs.restype = C.c_int
        L.sonar_batch_set_outputs.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                              P(sonar_ray_record), C.c_void_p]
        L.sonar_ping_batch.restype = C.c_int
        L.sonar_ping_batch.argtypes = [C.c_void_p, P(sonar_batch_plan), C.c_void_p, P(sonar_batch_options),
                                       C.c_void_p, C.c_size_t, C.c_void_p]
        L.sonar_batch_stamps.restype = C.c_int
        L.sonar_batch_stamps.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.sonar_batch_graph_create.restype = C.c_int
        L.sonar_batch_graph_create.argtypes = [C.c_void_p, P(sonar_batch_plan), C.c_void_p, P(sonar_batch_options),
                                               C.c_void_p, C.c_size_t, P(C.c_void_p)]
        L.sonar_graph_launch.restype = C.c_int
        L.sonar_graph_launch.argtypes = [C.c_void_p, C.c_void_p]
        L.sonar_graph_free.restype = None
        L.sonar_graph_free.argtypes = [C.c_void_p]
        L.sonar_batch_emit_desc_bytes.restype = C.c_size_t
        L.sonar_batch_emit_desc_bytes.argtypes = []
        L.sonar_batch_detect_workspace_size.restype = C.c_size_t
        L.sonar_batch_detect_workspace_size.argtypes = [C.c_int32, C.c_void_p]
        L.sonar_batch_prepare_detect.restype = C.c_int
        L.sonar_batch_prepare_detect.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, P(sonar_cfar), C.c_void_p,
                                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                                 C.c_void_p]
        L.sonar_batch_autotune.restype = C.c_int
        L.sonar_batch_autotune.argtypes = [C.c_void_p, P(sonar_batch_plan), C.c_void_p, C.c_void_p, C.c_size_t,
                                           C.c_void_p, P(sonar_batch_options), P(C.c_float)]
        L.sonar_surrogate_param_count.restype = C.c_int64
        L.sonar_surrogate_param_count.argtypes = []
        L.sonar_surrogate_create.restype = C.c_int
        L.sonar_surrogate_create.argtypes = [C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                             P(C.c_void_p)]
        L.sonar_surrogate_free.restype = None
        L.sonar_surrogate_free.argtypes = [C.c_void_p]
        L.sonar_surrogate_set_state.restype = C.c_int
        L.sonar_surrogate_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]
        L.sonar_surrogate_get_state.restype = C.c_int
        L.sonar_surrogate_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, P(C.c_int64)]
        L.sonar_surrogate_set_norm.restype = C.c_int
        L.sonar_surrogate_set_norm.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.sonar_surrogate_geometry.restype = C.c_int
        L.sonar_surrogate_geometry.argtypes = [P(sonar_params), P(sonar_pose), C.c_void_p]
        L.sonar_surrogate_forward.restype = C.c_int
        L.sonar_surrogate_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                              C.c_void_p, C.c_void_p]
        L.sonar_surrogate_train_step.restype = C.c_int
        L.sonar_surrogate_train_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                                 C.c_void_p, C.c_float, C.c_void_p, C.c_void_p]
        L.sonar_surrogate_gradient.restype = C.c_int
        L.sonar_surrogate_gradient.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.sonar_surrogate_set_loss_weights.restype = C.c_int
        L.sonar_surrogate_set_loss_weights.argtypes = [C.c_void_p, C.c_void_p]
        L.sonar_surrogate_target.restype = C.c_int
        L.sonar_surrogate_target.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                             C.c_void_p]
        L.sonar_surrogate_moments.restype = C.c_int
        L.sonar_surrogate_moments.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.sonar_surrogate_profile.restype = C.c_int
        L.sonar_surrogate_profile.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                              C.c_void_p, C.c_void_p, C.c_void_p]
        L.sonar_params_from_resolution.restype = C.c_int
        L.sonar_params_from_resolution.argtypes = [C.c_double] * 7 + [P(sonar_params)]
        L.sonar_ping_ssp.restype = C.c_int
        L.sonar_ping_ssp.argtypes = [C.c_void_p, P(sonar_params), P(sonar_pose), P(sonar_ssp), C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.sonar_ping_ssp_rx.restype = C.c_int
        L.sonar_ping_ssp_rx.argtypes = [C.c_void_p, P(sonar_params), P(sonar_pose), P(sonar_ssp), C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                        C.c_void_p]
        L.sonar_add_reverb.restype = C.c_int
        L.sonar_add_reverb.argtypes = [C.c_void_p, P(sonar_params), P(sonar_pose), P(sonar_reverb), C.c_void_p]
        L.sonar_rx_workspace_size.restype = C.c_size_t
        L.sonar_rx_workspace_size.argtypes = [P(sonar_params)]
        L.sonar_workspace_size.restype = C.c_size_t
        L.sonar_workspace_size.argtypes = [C.c_void_p, P(sonar_params), C.c_int32]
        L.sonar_ping_ws.restype = C.c_int
        L.sonar_ping_ws.argtypes = [C.c_void_p, P(sonar_params), P(sonar_pose), C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.sonar_ping_rx.restype = C.c_int
        L.sonar_ping_rx.argtypes = [C.c_void_p, P(sonar_params), P(sonar_pose), C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.sonar_pulse_dt.restype = C.c_int
        L.sonar_pulse_dt.argtypes = [P(sonar_params), P(sonar_pose), C.c_void_p, P(C.c_double)]
        L.sonar_lfm_pulse.restype = C.c_int
        L.sonar_lfm_pulse.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, C.c_void_p, C.c_int32,
                                      P(C.c_int32)]
        L.sonar_pulse_compress.restype = C.c_int
        L.sonar_pulse_compress.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                           C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _check(st):
    if st < 0:
        L = lib()
        raise SonarError(st, f"{L.sonar_status_string(st).decode()}: {L.sonar_last_error().decode()}")
    return st


def params_of(cfg) -> sonar_params:
    """sonar_params from a ``scenes.SensorConfig``."""
    return sonar_params(hfov=cfg.hfov, vfov=cfg.vfov, n_h=cfg.n_h, n_v=cfg.n_v, rays_per_beam=cfg.rays_per_beam,
                        grid_mode=cfg.grid_mode, jitter=cfg.jitter, n_range=cfg.n_range, r_min=cfg.r_min,
                        r_max=cfg.r_max, freq_hz=cfg.freq_hz, c0=cfg.c0, c_grad=cfg.c_grad,
                        abs_db_per_m=cfg.abs_db_per_m, max_bounces=cfg.max_bounces, pad0=0, k_d=cfg.k_d,
                        k_s=cfg.k_s, phong_n=cfg.phong_n, seed=cfg.seed, flags=cfg.flags, pad1=0)


def pose_of(pose) -> sonar_pose:
    q = sonar_pose()
    for i in range(3):
        q.position[i] = pose.position[i]
    for i in range(9):
        q.rot[i] = pose.rot[i]
    q.ping = pose.ping
    return q


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Scene:
    """A built scene (owns the library handle)."""

    def __init__(self, mesh, leaf_size: int = 0, stream=None, device_inputs: bool = False):
        import torch
        self._h = C.c_void_p()
        keep = []
        if device_inputs:
            arrs = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in
                    (mesh.vertices, mesh.indices, mesh.reflectivity, mesh.phase, mesh.material)]
            keep = arrs
            ptrs = [a.data_ptr() for a in arrs]
        else:
            arrs = [np.ascontiguousarray(a) for a in
                    (mesh.vertices.astype(np.float32), mesh.indices.astype(np.int32),
                     mesh.reflectivity.astype(np.float32), mesh.phase.astype(np.float32),
                     mesh.material.astype(np.uint8))]
            keep = arrs
            ptrs = [a.ctypes.data for a in arrs]
        m = sonar_mesh(vertices=ptrs[0], indices=ptrs[1], reflectivity=ptrs[2], phase=ptrs[3], material=ptrs[4],
                       n_vertices=int(mesh.vertices.shape[0]), n_triangles=int(mesh.indices.shape[0]),
                       on_device=1 if device_inputs else 0, leaf_size=leaf_size)
        _check(lib().sonar_build_scene(C.byref(m), _stream(stream), C.byref(self._h)))
        del keep

    def info(self) -> dict:
        i = sonar_scene_info()
        _check(lib().sonar_get_scene_info(self._h, C.byref(i)))
        return dict(n_triangles=i.n_triangles, n_nodes=i.n_nodes, depth=i.depth, leaf_size=i.leaf_size,
                    lo=list(i.lo), hi=list(i.hi), node_bytes=i.node_bytes, tri_bytes=i.tri_bytes)

    def status(self, stream=None) -> int:
        return lib().sonar_device_status(self._h, _stream(stream))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sonar_free_scene(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def beams_of(cfg):
    return (cfg.n_v + 1, cfg.n_h + 1) if cfg.grid_mode == 1 else (cfg.n_v, cfg.n_h)


def alloc_outputs(cfg, gbuffer=False, incoh=False, record=False, stats=False, device="cuda"):
    """Output tensors of a ping. ``record`` adds the per-ray record (with the
    retro-chain returns ``rbin`` / ``ramp`` under FLAG_RETRO_CHAIN and several
    bounces); ``stats`` (with ``record``) adds the traversal counters, which
    select the counting kernel instantiations."""
    import torch
    bv, bh = beams_of(cfg)
    out = dict(volume=torch.empty((bv, bh, cfg.n_range), dtype=torch.complex64, device=device))
    if gbuffer:
        out["gbuffer"] = torch.empty((bv, bh, 8), dtype=torch.float32, device=device)
    if incoh:
        out["incoh"] = torch.empty((2, bv, bh, cfg.n_range), dtype=torch.float32, device=device)
    if record:
        n = bv * bh * cfg.rays_per_beam
        K = cfg.max_bounces
        out["tri"] = torch.empty((n, K), dtype=torch.int32, device=device)
        out["bin"] = torch.empty((n, K), dtype=torch.int32, device=device)
        out["vis"] = torch.empty((n, K), dtype=torch.int32, device=device)
        out["amp"] = torch.empty((n, K), dtype=torch.complex64, device=device)
        out["beam"] = torch.empty((n, K), dtype=torch.int32, device=device)
        if (int(cfg.flags) & FLAG_RETRO_CHAIN) and K > 1:
            out["rbin"] = torch.empty((n, K), dtype=torch.int32, device=device)
            out["ramp"] = torch.empty((n, K), dtype=torch.complex64, device=device)
        if stats:
            out["stats"] = torch.empty((n, 3), dtype=torch.int32, device=device)
    return out


def _rx_workspace(out, p):
    """The receive-binning workspace, kept with the outputs (grown when too small)."""
    import torch
    need = lib().sonar_rx_workspace_size(C.byref(p))
    if need == 0:           # invalid parameters: the ping call reports why
        need = 256
    ws = out.get("rx_workspace")
    if ws is None or ws.numel() < need:
        ws = out["rx_workspace"] = torch.empty(need, dtype=torch.uint8, device=out["volume"].device)
    return ws


def _ping_workspace(scene, out, p):
    """The workspace of sonar_ping_ws, kept with the outputs (grown when too small)."""
    import torch
    need = max(lib().sonar_workspace_size(scene.handle, C.byref(p), 1), 256)
    ws = out.get("workspace")
    if ws is None or ws.numel() < need:
        ws = out["workspace"] = torch.empty(need, dtype=torch.uint8, device=out["volume"].device)
    return ws


def ping(scene: Scene, cfg, pose, out=None, gbuffer=False, incoh=False, record=False, ray_mask=None, stream=None,
         params=None, pose_s=None, stats=False, staged=False):
    """One ping; returns the dict of output tensors (allocated if ``out`` is None).
    ``staged``: through sonar_ping_ws with a workspace kept in ``out`` (several
    bounces run in stages)."""
    if out is None:
        out = alloc_outputs(cfg, gbuffer, incoh, record, stats)
    rec = None
    if "tri" in out:
        rec = sonar_ray_record(tri=out["tri"].data_ptr(), bin=out["bin"].data_ptr(), vis=out["vis"].data_ptr(),
                               amp=out["amp"].data_ptr(),
                               stats=out["stats"].data_ptr() if "stats" in out else None,
                               beam=out["beam"].data_ptr() if "beam" in out else None,
                               retro_bin=out["rbin"].data_ptr() if "rbin" in out else None,
                               retro_amp=out["ramp"].data_ptr() if "ramp" in out else None)
    p = params if params is not None else params_of(cfg)
    q = pose_s if pose_s is not None else pose_of(pose)
    if getattr(cfg, "ssp", ()):
        # piecewise-linear sound speed
        prof = ssp_of(cfg.ssp)
        if (p.flags & FLAG_RX_BEAMS) and p.max_bounces > 1:
            ws = _rx_workspace(out, p)
            _check(lib().sonar_ping_ssp_rx(scene.handle, C.byref(p), C.byref(q), C.byref(prof), _dptr(out["volume"]),
                                           _dptr(out.get("gbuffer")), _dptr(out.get("incoh")),
                                           C.byref(rec) if rec is not None else None, _dptr(ray_mask), _dptr(ws),
                                           ws.numel(), _stream(stream)))
            return out
        _check(lib().sonar_ping_ssp(scene.handle, C.byref(p), C.byref(q), C.byref(prof), _dptr(out["volume"]),
                                    _dptr(out.get("gbuffer")), _dptr(out.get("incoh")),
                                    C.byref(rec) if rec is not None else None, _dptr(ray_mask), _stream(stream)))
        return out
    if staged:
        ws = _ping_workspace(scene, out, p)
        _check(lib().sonar_ping_ws(scene.handle, C.byref(p), C.byref(q), _dptr(out["volume"]),
                                   _dptr(out.get("gbuffer")), _dptr(out.get("incoh")),
                                   C.byref(rec) if rec is not None else None, _dptr(ray_mask), _dptr(ws), ws.numel(),
                                   _stream(stream)))
        return out
    if (p.flags & FLAG_RX_BEAMS) and p.max_bounces > 1:
        ws = _rx_workspace(out, p)
        _check(lib().sonar_ping_rx(scene.handle, C.byref(p), C.byref(q), _dptr(out["volume"]),
                                   _dptr(out.get("gbuffer")), _dptr(out.get("incoh")),
                                   C.byref(rec) if rec is not None else None, _dptr(ray_mask), _dptr(ws), ws.numel(),
                                   _stream(stream)))
        return out
    _check(lib().sonar_ping(scene.handle, C.byref(p), C.byref(q), _dptr(out["volume"]), _dptr(out.get("gbuffer")),
                            _dptr(out.get("incoh")), C.byref(rec) if rec is not None else None, _dptr(ray_mask),
                            _stream(stream)))
    return out


class Detector:
    """CFAR detection with a preallocated workspace, points buffer and count."""

    def __init__(self, cfg, train=16, guard=4, max_per_beam=4, pfa=1e-4, noise_floor=1e-11, capacity=None):
        import torch
        self.cfg = cfg
        self.params = params_of(cfg)
        self.cfar = sonar_cfar(train=train, guard=guard, max_per_beam=max_per_beam, pad=0, pfa=pfa,
                               noise_floor=noise_floor)
        bv, bh = beams_of(cfg)
        self.capacity = capacity if capacity is not None else bv * bh * max_per_beam
        nbytes = lib().sonar_detect_workspace_size(C.byref(self.params))
        if nbytes == 0:
            _check(SONAR_E_INVALID)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.points = torch.empty((max(self.capacity, 1), 6), dtype=torch.int32, device="cuda")
        self.count = torch.zeros(1, dtype=torch.int32, device="cuda")

    def __call__(self, volume, pose, stream=None, pose_s=None):
        q = pose_s if pose_s is not None else pose_of(pose)
        st = lib().sonar_detect(_dptr(volume), C.byref(self.params), C.byref(q), C.byref(self.cfar),
                                _dptr(self.points), self.capacity, _dptr(self.count), _dptr(self.workspace),
                                self.workspace.numel(), _stream(stream))
        _check(st)
        return self.points, self.count

    def ping_detect(self, scene: "Scene", volume, pose, stream=None, pose_s=None):
        """Ping + detection with the CFAR test fused into the ping kernel."""
        if getattr(self.cfg, "ssp", ()):
            raise SonarError(SONAR_E_UNSUPPORTED, "layered profiles: call ping(), then the detector")
        q = pose_s if pose_s is not None else pose_of(pose)
        st = lib().sonar_ping_detect(scene.handle, C.byref(self.params), C.byref(q), C.byref(self.cfar),
                                     _dptr(volume), _dptr(self.points), self.capacity, _dptr(self.count),
                                     _dptr(self.workspace), self.workspace.numel(), _stream(stream))
        _check(st)
        return self.points, self.count

    def ping_detect_noalloc(self, scene: "Scene", volume, pose, stream=None, pose_s=None):
        """As ping_detect, through the allocation-free entry point (the
        library's per-GPU static scratch instead of this detector's workspace)."""
        q = pose_s if pose_s is not None else pose_of(pose)
        st = lib().sonar_ping_detect_noalloc(scene.handle, C.byref(self.params), C.byref(q), C.byref(self.cfar),
                                             _dptr(volume), _dptr(self.points), self.capacity, _dptr(self.count),
                                             _stream(stream))
        _check(st)
        return self.points, self.count

    def fetch(self):
        """Host copy of the detections as a structured array (synchronises)."""
        n = int(self.count.item())
        n = min(n, self.capacity)
        raw = self.points[:n].cpu().numpy()
        return raw.view(POINT_DTYPE).reshape(-1), int(self.count.item())


def params_from_resolution(hfov, vfov, dth_h, dth_v, r_min, r_max, dr, base=None) -> sonar_params:
    p = base if base is not None else sonar_params()
    _check(lib().sonar_params_from_resolution(hfov, vfov, dth_h, dth_v, r_min, r_max, dr, C.byref(p)))
    return p


MAX_PULSE_TAPS = 64


def add_reverb(volume, cfg, pose, sv_db: float, noise_power: float = 0.0, seed: int = 1, stream=None):
    """Adds water-column reverberation and receiver noise to a ping's volume in place."""
    rv = sonar_reverb(sv_db=float(sv_db), noise_power=float(noise_power), seed=int(seed))
    _check(lib().sonar_add_reverb(_dptr(volume), C.byref(params_of(cfg)), C.byref(pose_of(pose)), C.byref(rv),
                                  _stream(stream)))
    return volume


def pulse_dt(cfg, pose) -> float:
    """Two-way delay spacing of the range bins (sonar_pulse_dt)."""
    dt = C.c_double()
    prof = ssp_of(cfg.ssp) if getattr(cfg, "ssp", ()) else None
    _check(lib().sonar_pulse_dt(C.byref(params_of(cfg)), C.byref(pose_of(pose)),
                                C.byref(prof) if prof is not None else None, C.byref(dt)))
    return float(dt.value)


def lfm_pulse(bandwidth_hz: float, duration_s: float, dt_s: float, window: int = 0) -> np.ndarray:
    """Baseband linear-FM pulse sampled at dt (complex64), from the library."""
    taps = np.zeros(MAX_PULSE_TAPS, np.complex64)
    n = C.c_int32()
    _check(lib().sonar_lfm_pulse(float(bandwidth_hz), float(duration_s), float(dt_s), int(window), taps.ctypes.data,
                                 MAX_PULSE_TAPS, C.byref(n)))
    return taps[:n.value].copy()


def pulse_compress(volume, pulse, series=True, matched=True, out=None, stream=None):
    """Time series and matched-filter output of every beam column of a
    complex volume [..., n_bins] for a baseband pulse (complex taps)."""
    import torch
    n_bins = int(volume.shape[-1])
    n_beams = int(volume.numel() // max(n_bins, 1))
    p = np.ascontiguousarray(np.asarray(pulse, np.complex64))
    out = dict(out or {})
    if series and "series" not in out:
        out["series"] = torch.empty_like(volume)
    if matched and "matched" not in out:
        out["matched"] = torch.empty_like(volume)
    _check(lib().sonar_pulse_compress(_dptr(volume), n_beams, n_bins, p.ctypes.data, int(p.size),
                                      _dptr(out.get("series") if series else None),
                                      _dptr(out.get("matched") if matched else None), _stream(stream)))
    return out


class Graph:
    """An instantiated HIP graph of one batch launch."""

    def __init__(self, handle):
        self._h = handle

    def launch(self, stream=None):
        _check(lib().sonar_graph_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sonar_graph_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many pings (own pose, layout, rays per beam) in one persistent launch.

    ``items`` is a list of (SensorConfig, Pose). Output volumes are allocated
    here, one tensor per ping; descriptors live in device memory."""

    def __init__(self, scene: Scene, items):
        import torch
        n = len(items)
        profiles = {tuple(getattr(cfg, "ssp", ()) or ()) for cfg, _ in items}
        if len(profiles) > 1:
            raise SonarError(SONAR_E_INVALID, "the pings of a batch share one sound-speed profile")
        knots = profiles.pop()
        self.scene = scene
        self.items = items
        self.volumes = [alloc_outputs(cfg)["volume"] for cfg, _ in items]
        P = (sonar_params * n)(*[params_of(cfg) for cfg, _ in items])
        Q = (sonar_pose * n)(*[pose_of(p) for _, p in items])
        V = (C.c_void_p * n)(*[v.data_ptr() for v in self.volumes])
        db = lib().sonar_batch_desc_bytes()
        host = np.zeros(n * db, np.uint8)
        self.plan = sonar_batch_plan()
        self.rx_workspace = None
        rx_bytes = lib().sonar_batch_rx_workspace_size(n, P)
        if rx_bytes:
            # receive binning with several bounces: list areas per ping
            self.rx_workspace = torch.empty(rx_bytes, dtype=torch.uint8, device="cuda")
            prof = ssp_of(knots) if knots else None
            _check(lib().sonar_batch_prepare_rx(scene.handle, n, P, Q, C.byref(prof) if knots else None, V,
                                                _dptr(self.rx_workspace), rx_bytes, host.ctypes.data,
                                                C.byref(self.plan)))
        elif knots:
            prof = ssp_of(knots)
            _check(lib().sonar_batch_prepare_ssp(scene.handle, n, P, Q, C.byref(prof), V, host.ctypes.data,
                                                 C.byref(self.plan)))
        else:
            _check(lib().sonar_batch_prepare(scene.handle, n, P, Q, V, host.ctypes.data, C.byref(self.plan)))
        self._host, self._P, self._Q = host, P, Q
        self.desc = torch.from_numpy(host).cuda()
        self.workspace = torch.empty(lib().sonar_batch_workspace_size(n), dtype=torch.uint8, device="cuda")
        self.n = n
        self.emit = None

    def set_outputs(self, i, gbuffer=False, incoh=False, record=False, ray_mask=None):
        """Adds sonar_ping's optional outputs to ping i (G-buffer, incoherent
        channels, per-ray record; ``ray_mask``: device bit mask of rays that
        add nothing). Returns the dict of allocated tensors."""
        import torch
        cfg = self.items[i][0]
        out = alloc_outputs(cfg, gbuffer, incoh, record)
        del out["volume"]
        rec = None
        if record:
            rec = sonar_ray_record(tri=out["tri"].data_ptr(), bin=out["bin"].data_ptr(), vis=out["vis"].data_ptr(),
                                   amp=out["amp"].data_ptr(), stats=None, beam=out["beam"].data_ptr(),
                                   retro_bin=out["rbin"].data_ptr() if "rbin" in out else None,
                                   retro_amp=out["ramp"].data_ptr() if "ramp" in out else None)
        if ray_mask is not None:
            out["ray_mask"] = ray_mask
        _check(lib().sonar_batch_set_outputs(self._host.ctypes.data, self.n, i, _dptr(out.get("gbuffer")),
                                             _dptr(out.get("incoh")), C.byref(rec) if rec is not None else None,
                                             _dptr(ray_mask)))
        self.desc = torch.from_numpy(self._host).cuda()
        self.extras = getattr(self, "extras", {})
        self.extras[i] = out
        return out

    def detect(self, train=16, guard=4, max_per_beam=4, pfa=1e-4, noise_floor=1e-11):
        """Adds the point cloud of every ping: the CA-CFAR test in each ping's
        kernel and one batched emission after the pings (also in graphs)."""
        import torch
        n = self.n
        cf = sonar_cfar(train=train, guard=guard, max_per_beam=max_per_beam, pad=0, pfa=pfa, noise_floor=noise_floor)
        caps = [max(1, v.shape[0] * v.shape[1] * max_per_beam) for v in self.volumes]
        self.points = [torch.empty((c, 6), dtype=torch.int32, device="cuda") for c in caps]
        self.counts = torch.zeros(n, dtype=torch.int32, device="cuda")
        nbytes = lib().sonar_batch_detect_workspace_size(n, self._P)
        if nbytes == 0:
            _check(SONAR_E_INVALID)
        self.det_workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        PT = (C.c_void_p * n)(*[p.data_ptr() for p in self.points])
        CAP = (C.c_int32 * n)(*caps)
        emit = np.zeros(n * lib().sonar_batch_emit_desc_bytes(), np.uint8)
        _check(lib().sonar_batch_prepare_detect(n, self._P, self._Q, C.byref(cf), PT, CAP, _dptr(self.counts),
                                                _dptr(self.det_workspace), self.det_workspace.numel(),
                                                self._host.ctypes.data, emit.ctypes.data))
        self.desc = torch.from_numpy(self._host).cuda()
        self.emit = torch.from_numpy(emit).cuda()

    def point_cloud(self, i):
        """Points of ping i after a run (synchronises)."""
        c = int(self.counts[i].item())
        return self.points[i][:min(c, self.points[i].shape[0])].cpu().numpy().view(POINT_DTYPE).reshape(-1), c

    def options(self, blocks_per_cu=0, tiles_per_item=0, waves_per_block=0):
        return sonar_batch_options(blocks_per_cu=blocks_per_cu, tiles_per_item=tiles_per_item,
                                   emit_desc=self.emit.data_ptr() if self.emit is not None else None,
                                   waves_per_block=waves_per_block, pad=0)

    def run(self, options=None, stream=None):
        o = options if options is not None else self.options()
        _check(lib().sonar_ping_batch(self.scene.handle, C.byref(self.plan), _dptr(self.desc), C.byref(o),
                                      _dptr(self.workspace), self.workspace.numel(), _stream(stream)))

    def graph(self, options=None) -> Graph:
        o = options if options is not None else self.options()
        h = C.c_void_p()
        _check(lib().sonar_batch_graph_create(self.scene.handle, C.byref(self.plan), _dptr(self.desc), C.byref(o),
                                              _dptr(self.workspace), self.workspace.numel(), C.byref(h)))
        return Graph(h)

    def autotune(self, stream=None):
        """Fastest launch knobs for the pings (timed without the emission);
        returns options that include this batch's emission if it has one."""
        best = sonar_batch_options()
        ms = C.c_float()
        _check(lib().sonar_batch_autotune(self.scene.handle, C.byref(self.plan), _dptr(self.desc),
                                          _dptr(self.workspace), self.workspace.numel(), _stream(stream),
                                          C.byref(best), C.byref(ms)))
        return self.options(best.blocks_per_cu, best.tiles_per_item, best.waves_per_block), float(ms.value)

    def stamps(self, stream=None):
        """(start, finish) device clock stamps per ping, 100 MHz ticks."""
        a = np.zeros(self.n, np.uint64)
        b = np.zeros(self.n, np.uint64)
        _check(lib().sonar_batch_stamps(_dptr(self.workspace), self.n, a.ctypes.data, b.ctypes.data, _stream(stream)))
        return a, b


def surrogate_geometry(cfg, poses):
    """Host float32 [len(poses), 16]: the surrogate's geometry block of each
    pose (sonar_surrogate_geometry)."""
    p = params_of(cfg)
    out = np.zeros((len(poses), 16), np.float32)
    for i, pose in enumerate(poses):
        q = pose_of(pose)
        _check(lib().sonar_surrogate_geometry(C.byref(p), C.byref(q), out[i].ctypes.data))
    return out


def _geo_check(geo, n):
    if tuple(geo.shape) != (n, 16) or not geo.is_contiguous():
        raise ValueError(f"geometry must be a contiguous [{n}, 16] tensor, got {tuple(geo.shape)}")


class Surrogate:
    """The learned multipath surrogate (weights, Adam state, activations on the device)."""

    def __init__(self, max_rows: int, n_bins: int, r_min: float = 0.3, r_max: float = 15.0, smooth: int = 32):
        self._h = C.c_void_p()
        _check(lib().sonar_surrogate_create(int(max_rows), int(n_bins), float(r_min), float(r_max), int(smooth),
                                            C.byref(self._h)))
        self.n_params = int(lib().sonar_surrogate_param_count())
        self.n_bins = n_bins
        self.max_rows = max_rows

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sonar_surrogate_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, params, adam_m=None, adam_v=None, step=0):
        p = np.ascontiguousarray(params, np.float32)
        m = None if adam_m is None else np.ascontiguousarray(adam_m, np.float32)
        v = None if adam_v is None else np.ascontiguousarray(adam_v, np.float32)
        _check(lib().sonar_surrogate_set_state(self._h, p.ctypes.data, m.ctypes.data if m is not None else None,
                                               v.ctypes.data if v is not None else None, int(step)))

    def get_state(self):
        n = self.n_params
        p, m, v = (np.zeros(n, np.float32) for _ in range(3))
        st = C.c_int64()
        _check(lib().sonar_surrogate_get_state(self._h, p.ctypes.data, m.ctypes.data, v.ctypes.data, C.byref(st)))
        return p, m, v, int(st.value)

    def set_norm(self, mean, std):
        a = np.ascontiguousarray(mean, np.float32)
        b = np.ascontiguousarray(std, np.float32)
        _check(lib().sonar_surrogate_set_norm(self._h, a.ctypes.data, b.ctypes.data))
        self.mean, self.std = a, b

    def forward(self, gbuf, geo, out=None, stream=None):
        """`gbuf` [n, H, W, 8] and `geo` [n, 16] (surrogate_geometry) on the device."""
        import torch
        n, H, W = gbuf.shape[0], gbuf.shape[1], gbuf.shape[2]
        _geo_check(geo, n)
        out = out if out is not None else torch.empty((n * H * W, 64), dtype=torch.float32, device="cuda")
        _check(lib().sonar_surrogate_forward(self._h, _dptr(gbuf), _dptr(geo), n, H, W, _dptr(out), _stream(stream)))
        return out

    def train_step(self, gbuf, geo, target, lr, loss_out, stream=None):
        n, H, W = gbuf.shape[0], gbuf.shape[1], gbuf.shape[2]
        _geo_check(geo, n)
        _check(lib().sonar_surrogate_train_step(self._h, _dptr(gbuf), _dptr(geo), n, H, W, _dptr(target), float(lr),
                                                _dptr(loss_out), _stream(stream)))

    def gradient(self, gbuf, geo, target, stream=None):
        import torch
        n, H, W = gbuf.shape[0], gbuf.shape[1], gbuf.shape[2]
        _geo_check(geo, n)
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().sonar_surrogate_gradient(self._h, _dptr(gbuf), _dptr(geo), n, H, W, _dptr(target), _dptr(g),
                                              _dptr(loss), _stream(stream)))
        return g, loss

    def set_loss_weights(self, w=None):
        a = None if w is None else np.ascontiguousarray(w, np.float32)
        _check(lib().sonar_surrogate_set_loss_weights(self._h, a.ctypes.data if a is not None else None))

    def target(self, im, gbuf, standardize=True, out=None, stream=None):
        """Level-target coefficients [rows, 64] of the later-bounce channel `im`."""
        import torch
        rows = im.numel() // self.n_bins
        out = out if out is not None else torch.empty((rows, 64), dtype=torch.float32, device="cuda")
        _check(lib().sonar_surrogate_target(self._h, _dptr(im), _dptr(gbuf), rows, 1 if standardize else 0,
                                            _dptr(out), _stream(stream)))
        return out

    def moments(self, coef, stream=None):
        s1 = np.zeros(64)
        s2 = np.zeros(64)
        _check(lib().sonar_surrogate_moments(self._h, _dptr(coef), coef.shape[0], s1.ctypes.data, s2.ctypes.data,
                                             _stream(stream)))
        return s1, s2

    def profile(self, coef, i1, gbuf, im=None, want_profile=True, stream=None, out=None):
        """Predicted profile [rows, n_bins] (into `out` if given) and, with `im`,
        the per-beam errors [rows, 8]."""
        import torch
        rows = coef.shape[0]
        prof = None
        if want_profile:
            prof = out if out is not None else torch.empty((rows, self.n_bins), dtype=torch.float32, device="cuda")
        err = torch.empty((rows, 8), dtype=torch.float32, device="cuda") if im is not None else None
        _check(lib().sonar_surrogate_profile(self._h, _dptr(coef), _dptr(i1), _dptr(im), _dptr(gbuf), rows,
                                             _dptr(prof), _dptr(err), _stream(stream)))
        return prof, err
