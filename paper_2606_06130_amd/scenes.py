"""Seeded synthetic inputs: triangle meshes, per-facet materials, sensor poses
and sensor configurations.

This module holds no part of the echo model's arithmetic. It only produces the
arrays that both the HIP path and the CPU oracle consume, so that the two sides
see identical FP32 vertices, int32 indices and per-facet coefficients.

Workloads (synthetic stand-ins for the paper's scenes, Sec. IV and Sec. V):
  * ``scene_seabed_boxes``: a 20 x 20 m seabed at z = -10 m tessellated as
    32 x 32 quads plus 8 open-bottom boxes (2,128 triangles).
  * ``scene_harbor``: a corrugated sheet-pile wall (trapezoidal profile, period
    1.2 m, depth 0.3 m, front face at x = 6 m, 30 m long, 12 m tall) over a
    512 x 512 fBm heightfield seabed (601,088 triangles); Sec. V-A motivates it.
  * ``scene_harbor_multipath``: the harbor scene plus a pressure-release water
    surface at z = +2 m and 50 open cylinders as piles (1,991,680 triangles).

Material codes: 0 = rough facet, 1 = pressure-release surface.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MAT_ROUGH = 0
MAT_PRESSURE_RELEASE = 1


@dataclass
class Mesh:
    vertices: np.ndarray      # float32 [n_v, 3], world metres, z up
    indices: np.ndarray       # int32 [T, 3]
    reflectivity: np.ndarray  # float32 [T], intensity coefficient rho
    phase: np.ndarray         # float32 [T], per-facet phase in [0, 2*pi)
    material: np.ndarray      # uint8 [T]
    name: str = ""

    @property
    def n_triangles(self) -> int:
        return int(self.indices.shape[0])

    @property
    def n_vertices(self) -> int:
        return int(self.vertices.shape[0])


@dataclass
class Pose:
    position: tuple          # 3 floats, world metres
    rot: tuple               # 9 floats, row-major sensor->world; columns are sensor x (fwd), y (left), z (up)
    ping: int = 0            # ping counter, part of the jitter counter

    def as_arrays(self):
        return (np.asarray(self.position, np.float64), np.asarray(self.rot, np.float64).reshape(3, 3))


@dataclass
class SensorConfig:
    hfov: float = math.radians(90.0)
    vfov: float = math.radians(40.0)
    n_h: int = 64
    n_v: int = 32
    rays_per_beam: int = 4
    grid_mode: int = 0        # 0: cell-centred beams with stratified jitter, 1: LiDAR firing grid
    jitter: int = 1
    r_min: float = 0.3
    r_max: float = 15.0
    n_range: int = 256
    freq_hz: float = 1.0e6
    c0: float = 1500.0
    c_grad: float = 0.0       # c(z) = c0 + c_grad * z
    abs_db_per_m: float = 0.3
    max_bounces: int = 1
    k_d: float = 1.0
    k_s: float = 0.0
    phong_n: float = 20.0
    seed: int = 1000
    flags: int = 0
    ssp: tuple = ()           # knots (z, c) of a piecewise-linear sound speed (replaces c0, c_grad), or ()
    extra: dict = field(default_factory=dict)

    @property
    def n_beams(self) -> int:
        if self.grid_mode == 1:
            return (self.n_h + 1) * (self.n_v + 1)
        return self.n_h * self.n_v

    @property
    def n_rays(self) -> int:
        return self.n_beams * self.rays_per_beam

    def replace(self, **kw) -> "SensorConfig":
        d = dict(self.__dict__)
        d.update(kw)
        return SensorConfig(**d)


# ----------------------------------------------------------------------------
# rotations and poses


def rot_ypr(yaw: float, pitch_down: float, roll: float) -> tuple:
    """Sensor->world rotation R = Rz(yaw) Ry(pitch_down) Rx(roll), row-major.

    A positive ``pitch_down`` tilts the sensor's forward axis below the horizon.
    """
    cy, sy = math.cos(yaw), math.sin(yaw)
    cp, sp = math.cos(pitch_down), math.sin(pitch_down)
    cr, sr = math.cos(roll), math.sin(roll)
    rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]], np.float64)
    ry = np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]], np.float64)
    rx = np.array([[1, 0, 0], [0, cr, -sr], [0, sr, cr]], np.float64)
    r = rz @ ry @ rx
    return tuple(float(x) for x in r.reshape(-1))


def pose(position, yaw=0.0, pitch_down=0.0, roll=0.0, ping=0) -> Pose:
    return Pose(tuple(float(x) for x in position), rot_ypr(yaw, pitch_down, roll), ping)


# ----------------------------------------------------------------------------
# mesh builders


def _grid(x0, x1, y0, y1, nx, ny, zfun):
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")        # [ny+1, nx+1]
    Z = zfun(X, Y)
    verts = np.stack([X, Y, Z], -1).reshape(-1, 3)
    i = np.arange(ny)[:, None]
    j = np.arange(nx)[None, :]
    a = i * (nx + 1) + j
    b = a + 1
    c = a + (nx + 1)
    d = c + 1
    t1 = np.stack([a, b, d], -1).reshape(-1, 3)
    t2 = np.stack([a, d, c], -1).reshape(-1, 3)
    tris = np.stack([t1, t2], 1).reshape(-1, 3)
    return verts, tris


def _box(cx, cy, z0, ex, ey, ez):
    """Axis-aligned box standing on z0 with no bottom face: 5 faces, 10 triangles."""
    x0, x1 = cx - ex / 2, cx + ex / 2
    y0, y1 = cy - ey / 2, cy + ey / 2
    z1 = z0 + ez
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], np.float64)
    quads = [(4, 5, 6, 7),            # top
             (0, 1, 5, 4),            # y0 side
             (1, 2, 6, 5),            # x1 side
             (2, 3, 7, 6),            # y1 side
             (3, 0, 4, 7)]            # x0 side
    t = []
    for a, b, c, d in quads:
        t.append((a, b, c))
        t.append((a, c, d))
    return v, np.array(t, np.int64)


def _cylinder(cx, cy, r, z0, z1, nseg, nrows):
    """Open cylinder (no caps): nseg x nrows quads, 2 * nseg * nrows triangles."""
    ang = np.arange(nseg) * (2 * math.pi / nseg)
    zs = np.linspace(z0, z1, nrows + 1)
    A, Z = np.meshgrid(ang, zs, indexing="xy")       # [nrows+1, nseg]
    verts = np.stack([cx + r * np.cos(A), cy + r * np.sin(A), Z], -1).reshape(-1, 3)
    i = np.arange(nrows)[:, None]
    j = np.arange(nseg)[None, :]
    a = i * nseg + j
    b = i * nseg + (j + 1) % nseg
    c = a + nseg
    d = b + nseg
    t1 = np.stack([a, b, d], -1).reshape(-1, 3)
    t2 = np.stack([a, d, c], -1).reshape(-1, 3)
    return verts, np.stack([t1, t2], 1).reshape(-1, 3)


def _sheet_pile_wall(x_front, y0, y1, z0, z1, period, flange, web, depth, nrows):
    """Corrugated wall: the plan-view profile x(y) is a trapezoid wave.

    One period is a front flange (x = x_front), a web moving away from the
    sensor by ``depth``, a back flange and a web returning. Each straight run is
    one vertical strip of ``nrows`` quads.
    """
    n_per = int(round((y1 - y0) / period))
    ys = [y0]
    xs = [x_front]
    for p in range(n_per):
        base = y0 + p * period
        for dy, x in ((flange, x_front), (flange + web, x_front + depth),
                      (2 * flange + web, x_front + depth), (period, x_front)):
            ys.append(base + dy)
            xs.append(x)
    ys = np.array(ys)
    xs = np.array(xs)
    ncol = len(ys)                                   # 4 * n_per + 1 profile points
    zs = np.linspace(z0, z1, nrows + 1)
    Y, Z = np.meshgrid(ys, zs, indexing="xy")
    X, _ = np.meshgrid(xs, zs, indexing="xy")
    verts = np.stack([X, Y, Z], -1).reshape(-1, 3)
    i = np.arange(nrows)[:, None]
    j = np.arange(ncol - 1)[None, :]
    a = i * ncol + j
    b = a + 1
    c = a + ncol
    d = c + 1
    t1 = np.stack([a, b, d], -1).reshape(-1, 3)
    t2 = np.stack([a, d, c], -1).reshape(-1, 3)
    return verts, np.stack([t1, t2], 1).reshape(-1, 3)


def _lattice_hash(ix, iy, octave, seed):
    """Integer hash of a lattice point -> uniform in [-1, 1] (SplitMix64 finaliser)."""
    m = np.uint64(0xFFFFFFFFFFFFFFFF)
    z = (np.asarray(ix, np.int64).astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
         ^ np.asarray(iy, np.int64).astype(np.uint64) * np.uint64(0xC2B2AE3D27D4EB4F)
         ^ np.uint64((seed * 1000003 + octave * 7919) & 0xFFFFFFFFFFFFFFFF))
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9) & m
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB) & m
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 / 2.0**53) - 1.0


def fbm_height(x, y, seed, octaves=4, base_freq=0.25, lacunarity=2.0, gain=0.5, amplitude=0.5):
    """Value-noise fBm on a unit lattice with smoothstep interpolation.

    Octave o samples at frequency base_freq * lacunarity**o with weight gain**o;
    the sum is scaled so its largest possible magnitude equals ``amplitude``.
    """
    total = np.zeros_like(x, dtype=np.float64)
    wsum = 0.0
    for o in range(octaves):
        f = base_freq * lacunarity ** o
        w = gain ** o
        qx, qy = x * f, y * f
        ix, iy = np.floor(qx), np.floor(qy)
        fx, fy = qx - ix, qy - iy
        sx = fx * fx * (3 - 2 * fx)
        sy = fy * fy * (3 - 2 * fy)
        ix = ix.astype(np.int64)
        iy = iy.astype(np.int64)
        h00 = _lattice_hash(ix, iy, o, seed)
        h10 = _lattice_hash(ix + 1, iy, o, seed)
        h01 = _lattice_hash(ix, iy + 1, o, seed)
        h11 = _lattice_hash(ix + 1, iy + 1, o, seed)
        v = (h00 * (1 - sx) + h10 * sx) * (1 - sy) + (h01 * (1 - sx) + h11 * sx) * sy
        total += w * v
        wsum += w
    return total * (amplitude / wsum)


def _assemble(parts, rng, name, surface_parts=()):
    """Concatenate (verts, tris) parts; draw rho ~ U[0.1, 0.9] and phase ~ U[0, 2pi)
    per facet. ``surface_parts`` are pressure-release: rho = 1, phase = 0."""
    vs, ts, mats = [], [], []
    off = 0
    for k, (v, t) in enumerate(list(parts) + list(surface_parts)):
        vs.append(v)
        ts.append(t + off)
        off += v.shape[0]
        mats.append(np.full(t.shape[0], MAT_PRESSURE_RELEASE if k >= len(parts) else MAT_ROUGH, np.uint8))
    verts = np.concatenate(vs).astype(np.float32)
    tris = np.concatenate(ts).astype(np.int32)
    mat = np.concatenate(mats)
    T = tris.shape[0]
    rho = rng.uniform(0.1, 0.9, T).astype(np.float32)
    phi = rng.uniform(0.0, 2 * math.pi, T).astype(np.float32)
    surf = mat == MAT_PRESSURE_RELEASE
    rho[surf] = 1.0
    phi[surf] = 0.0
    return Mesh(verts, tris, rho, phi, mat, name)


# ----------------------------------------------------------------------------
# the three scenes


def scene_seabed_boxes(seed: int = 1) -> Mesh:
    """Flat 20 x 20 m seabed at z = -10 m (x in [0, 20], y in [-10, 10], 32 x 32
    quads) plus 8 axis-aligned open-bottom boxes with edges U[0.5, 2] m placed
    uniformly on it: 2,048 + 80 = 2,128 triangles."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [_grid(0.0, 20.0, -10.0, 10.0, 32, 32, lambda X, Y: np.full_like(X, -10.0))]
    for _ in range(8):
        ex, ey, ez = rng.uniform(0.5, 2.0, 3)
        cx = rng.uniform(ex / 2, 20.0 - ex / 2)
        cy = rng.uniform(-10.0 + ey / 2, 10.0 - ey / 2)
        parts.append(_box(cx, cy, -10.0, ex, ey, ez))
    return _assemble(parts, rng, "seabed_boxes")


def _harbor_parts(seed):
    seabed = _grid(-9.0, 21.0, -15.0, 15.0, 512, 512,
                   lambda X, Y: -10.0 + fbm_height(X, Y, seed))
    wall = _sheet_pile_wall(6.0, -15.0, 15.0, -10.0, 2.0, 1.2, 0.4, 0.2, 0.3, 384)
    return [seabed, wall]


def scene_harbor(seed: int = 2) -> Mesh:
    """Sheet-pile wall over an fBm seabed: 524,288 + 76,800 = 601,088 triangles."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return _assemble(_harbor_parts(seed), rng, "harbor")


def pile_centres(seed: int = 3, n: int = 50):
    """50 pile centres uniform in x in [-8, 5.2], y in [-14, 14], at least 1 m
    apart and at least 1.5 m from the origin (rejection sampling)."""
    rng = np.random.Generator(np.random.PCG64(seed * 7 + 11))
    out = []
    while len(out) < n:
        x, y = rng.uniform(-8.0, 5.2), rng.uniform(-14.0, 14.0)
        if math.hypot(x, y) < 1.5:
            continue
        if any(math.hypot(x - a, y - b) < 1.0 for a, b, _ in out):
            continue
        out.append((x, y, rng.uniform(0.15, 0.4)))
    return out


def scene_harbor_multipath(seed: int = 3) -> Mesh:
    """Harbor scene + water surface at z = +2 m (64 x 64 quads, pressure-release)
    + 50 open cylinders (128 segments x 108 rows, z in [-10.5, 2]):
    601,088 + 8,192 + 1,382,400 = 1,991,680 triangles."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = _harbor_parts(seed)
    for x, y, r in pile_centres(seed):
        parts.append(_cylinder(x, y, r, -10.5, 2.0, 128, 108))
    surface = _grid(-9.0, 21.0, -15.0, 15.0, 64, 64, lambda X, Y: np.full_like(X, 2.0))
    return _assemble(parts, rng, "harbor_multipath", surface_parts=[surface])


# ----------------------------------------------------------------------------
# sensor configurations and poses of the five workloads


def sensor_seabed_boxes() -> SensorConfig:
    """90 x 40 deg FOV, 64 x 32 beams, 4 jittered rays per beam, 0.3-15 m in 256
    bins, c = 1500 m/s, 1 MHz, 0.3 dB/m, single bounce, Lambert cos^2."""
    return SensorConfig()


def pose_seabed_boxes() -> Pose:
    """Sensor at the origin, boresight pitched 60 deg down so that the seabed
    lies at about 10-15 m."""
    return pose((0.0, 0.0, 0.0), pitch_down=math.radians(60.0))


def pose_seabed_boxes_level() -> Pose:
    """Sensor at the origin looking along +x with no pitch: every ray stays above
    z = -15 sin(20 deg) within 15 m, so the volume is empty."""
    return pose((0.0, 0.0, 0.0))


def sensor_harbor() -> SensorConfig:
    """256 x 128 beams x 16 jittered rays (524,288 rays), 1,024 bins to 15 m,
    single bounce."""
    return SensorConfig(n_h=256, n_v=128, rays_per_beam=16, n_range=1024)


def pose_harbor() -> Pose:
    """Inspection pose facing the wall: 3 m below the surface datum, pitched
    35 deg down, so the view holds the wall and the seabed in front of it."""
    return pose((0.0, 0.0, -3.0), pitch_down=math.radians(35.0))


def sensor_harbor_multipath() -> SensorConfig:
    """Harbor sensor with 3 bounces, Phong-20 lobe plus diffuse (k_d 0.7, k_s 0.3)
    and c(z) = 1500 + 0.05 z."""
    return SensorConfig(n_h=256, n_v=128, rays_per_beam=16, n_range=1024, max_bounces=3,
                        k_d=0.7, k_s=0.3, phong_n=20.0, c_grad=0.05)


BATCH_LAYOUTS = ((64, 32), (128, 64), (256, 128))
BATCH_RAYS = (4, 8, 16)


def lawnmower_batch(seed: int = 4, n_pings: int = 256):
    """256 pings on a boustrophedon path: 4 lanes at z in {-1, -3, -5, -7} m,
    x = 0, y sweeping +-12 m, 64 poses per lane, heading +x; N(0, 0.1 m) position
    and N(0, 2 deg) yaw/pitch/roll jitter; beam layout and rays per beam drawn
    uniformly. Returns a list of (SensorConfig, Pose)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = sensor_harbor_multipath()
    out = []
    per_lane = n_pings // 4
    for p in range(n_pings):
        lane, k = divmod(p, per_lane)
        z = (-1.0, -3.0, -5.0, -7.0)[lane % 4]
        t = k / max(per_lane - 1, 1)
        y = -12.0 + 24.0 * t if lane % 2 == 0 else 12.0 - 24.0 * t
        pos = np.array([0.0, y, z]) + rng.normal(0.0, 0.1, 3)
        yaw, pitch, roll = rng.normal(0.0, math.radians(2.0), 3)
        li = int(rng.integers(0, 3))
        nr = int(BATCH_RAYS[int(rng.integers(0, 3))])
        nh, nv = BATCH_LAYOUTS[li]
        cfg = base.replace(n_h=nh, n_v=nv, rays_per_beam=nr)
        out.append((cfg, pose(pos, yaw, pitch + math.radians(20.0), roll, ping=p)))
    return out


def random_poses(seed: int, n: int, pile_seed: int = 3):
    """Random survey poses: x in [-6, 4], y in [-12, 12], z in [-8, 0.5], yaw
    U[-60, 60] deg, pitch U[-30, 15] deg (positive looks up), roll 0; poses
    within 0.75 m of a pile or 0.5 m of the seabed or surface are rejected."""
    rng = np.random.Generator(np.random.PCG64(seed))
    piles = pile_centres(pile_seed)
    out = []
    while len(out) < n:
        x, y, z = rng.uniform(-6, 4), rng.uniform(-12, 12), rng.uniform(-8, 0.5)
        yaw = math.radians(rng.uniform(-60, 60))
        pitch_up = math.radians(rng.uniform(-30, 15))
        if any(math.hypot(x - a, y - b) < r + 0.75 for a, b, r in piles):
            continue
        if z < -10.5 + 0.5 + 0.5 or z > 2.0 - 0.5:
            continue
        out.append(pose((x, y, z), yaw, -pitch_up, 0.0, ping=len(out)))
    return out


# ----------------------------------------------------------------------------
# initial weights of the multipath surrogate (random draws shared by the
# library and its checks)

SURROGATE_LAYERS = ((174, 64), (64, 256), (256, 256), (256, 256), (256, 64))


def surrogate_init_params(seed: int) -> np.ndarray:
    """He-uniform weights U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)) and zero
    biases, in the parameter-vector layout (per layer W [fan_in][fan_out] then b)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for k, n in SURROGATE_LAYERS:
        lim = math.sqrt(6.0 / k)
        parts.append(rng.uniform(-lim, lim, k * n))
        parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)
