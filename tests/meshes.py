"""Small hand-built meshes for closed-form checks (test inputs only)."""
import math

import numpy as np

from paper_2606_06130_amd.scenes import Mesh, MAT_ROUGH, MAT_PRESSURE_RELEASE


def mesh_from(tris, rho=0.5, phi=0.0, mat=MAT_ROUGH):
    tris = np.asarray(tris, np.float64).reshape(-1, 3, 3)
    T = tris.shape[0]
    v = tris.reshape(-1, 3).astype(np.float32)
    idx = np.arange(3 * T, dtype=np.int32).reshape(T, 3)

    def arr(x, dt):
        a = np.asarray(x, dt)
        return np.full(T, a, dt) if a.ndim == 0 else a.astype(dt)
    return Mesh(v, idx, arr(rho, np.float32), arr(phi, np.float32), arr(mat, np.uint8), "test")


def concat(*meshes):
    v, i, r, p, m = [], [], [], [], []
    off = 0
    for me in meshes:
        v.append(me.vertices)
        i.append(me.indices + off)
        off += me.vertices.shape[0]
        r.append(me.reflectivity)
        p.append(me.phase)
        m.append(me.material)
    return Mesh(np.concatenate(v), np.concatenate(i).astype(np.int32), np.concatenate(r),
                np.concatenate(p), np.concatenate(m), "test")


def big_triangle_x(x, half=300.0):
    """One triangle in the plane x = const that covers |y|, |z| < half / 2."""
    return [[x, -half, -half], [x, half, -half], [x, 0.0, 2 * half]]


def big_triangle_z(z, half=300.0):
    return [[-half, -half, z], [half, -half, z], [0.0, 2 * half, z]]


def icosphere(centre, radius, subdiv):
    t = (1 + 5 ** 0.5) / 2
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
             (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = [np.array(v, np.float64) / np.linalg.norm(v) for v in verts]
    F = faces
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]
        nf = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    V = np.array(V) * radius + np.asarray(centre, np.float64)
    return V.astype(np.float32), np.array(F, np.int32)


def plane_grid_x(x, y0, y1, z0, z1, n, rng):
    ys = np.linspace(y0, y1, n + 1)
    zs = np.linspace(z0, z1, n + 1)
    Y, Z = np.meshgrid(ys, zs, indexing="xy")
    V = np.stack([np.full_like(Y, x), Y, Z], -1).reshape(-1, 3)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    a = i * (n + 1) + j
    tri = np.concatenate([np.stack([a, a + 1, a + n + 2], -1).reshape(-1, 3),
                          np.stack([a, a + n + 2, a + n + 1], -1).reshape(-1, 3)])
    T = tri.shape[0]
    return Mesh(V.astype(np.float32), tri.astype(np.int32), np.full(T, 0.5, np.float32),
                rng.uniform(0, 2 * math.pi, T).astype(np.float32), np.zeros(T, np.uint8), "grid")


def deep_chain(levels=20, per_level=64, size=2.0, length=2.0, wall_x=-1.0):
    """A hierarchy that forces deep traversal stacks. Clusters of `per_level`
    identical sliver triangles lie in the planes x = length (1 - 2^-i),
    i = 0 .. levels - 1; each sliver fills y + z < -size / 2 inside the square
    [-size, size / 2]^2, so its box contains the x axis while the triangle
    keeps clear of it by at least size / 2. A wall triangle at x = wall_x ends
    the rays. The geometric positions split one cluster off per Morton bit, so
    the hierarchy is a chain of balanced cluster subtrees, and a ray running
    down the axis toward -x enters every box on the chain with the rest of the
    chain as the near child: it pushes one far child per level."""
    tris = []
    for i in range(levels):
        x = length * (1.0 - 2.0 ** -i)
        sl = [[x, -size, size / 2], [x, size / 2, -size], [x, -size, -size]]
        tris.extend([sl] * per_level)
    tris.append(big_triangle_x(wall_x, half=40.0))
    return mesh_from(tris, rho=0.5, phi=0.25)
