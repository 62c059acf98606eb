"""An independent ray shooter for piecewise-linear sound-speed profiles, used
to pin the oracle's eigenrays (CPU only).

In a layer with c(z) = c0 + g z a ray is a circle centred on the depth where
c would vanish (Sec. II-A: rays bend by Snell's law); this walker follows those
circles geometrically in the vertical plane of a ray, layer by layer, from a
start depth and grazing angle until a horizontal distance D. Travel time is
integrated numerically along each arc (Gauss-Legendre), not taken from a
closed form. Shooting a fan of angles and bracketing the depth mismatch at D
gives every eigenray between two points, turning or not."""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq

_GL_X, _GL_W = np.polynomial.legendre.leggauss(24)


class Profile:
    def __init__(self, knots):
        self.z = np.array([k[0] for k in knots], float)
        self.c = np.array([k[1] for k in knots], float)
        self.g = np.diff(self.c) / np.diff(self.z)
        self.n = len(self.g)

    def layer(self, z, up):
        """Layer holding depth z for a ray going up (a knot belongs to the
        layer above) or down (the layer below)."""
        i = int(np.searchsorted(self.z, z, side="right")) - 1
        i = min(max(i, 0), self.n - 1)
        if not up and i > 0 and z == self.z[i]:
            i -= 1
        return i

    def speed(self, i, z):
        return self.c[i] + self.g[i] * (z - self.z[i])


def _arc_time(g, psi0, psi1, n_sub=4):
    """(1 / |g|) * integral of sec(psi) over [psi0, psi1], by quadrature."""
    total = 0.0
    edges = np.linspace(psi0, psi1, n_sub + 1)
    for a, b in zip(edges[:-1], edges[1:]):
        x = 0.5 * (b - a) * _GL_X + 0.5 * (a + b)
        total += 0.5 * (b - a) * float(np.sum(_GL_W / np.cos(x)))
    return total / abs(g)


def walk(prof: Profile, z0: float, theta0: float, D: float, max_pieces: int = 200):
    """Follow the ray from (0, z0) at grazing angle theta0 (positive up) to
    horizontal distance D. Returns (z, theta, T, L) there."""
    x, z, th, T, L = 0.0, z0, theta0, 0.0, 0.0
    up = th > 0.0
    for _ in range(max_pieces):
        i = prof.layer(z, up)
        g = prof.g[i]
        top = prof.z[i + 1] if i + 1 < prof.n else math.inf
        bot = prof.z[i] if i > 0 else -math.inf
        if g == 0.0:
            c = prof.speed(i, z)
            zb = top if th > 0 else (bot if th < 0 else None)
            xe = x + (zb - z) / math.tan(th) if zb is not None and math.isfinite(zb) else math.inf
            if xe >= D:
                ds = (D - x) / math.cos(th)
                return z + (D - x) * math.tan(th), th, T + ds / c, L + ds
            ds = (xe - x) / math.cos(th)
            x, z, T, L = xe, zb, T + ds / c, L + ds
            up = th > 0.0
            continue
        c0 = prof.c[i] - g * prof.z[i]
        zc = -c0 / g                              # the depth where c would vanish
        sg = 1.0 if g > 0 else -1.0
        t = (zc - z) / math.cos(th)
        xc = x - t * math.sin(th)
        R = abs(t)
        psi0 = math.atan2(x - xc, sg * (z - zc))
        cands = []
        for zb in (top, bot):
            if not math.isfinite(zb):
                continue
            cp = sg * (zb - zc) / R
            if abs(cp) <= 1.0:
                for p in (math.acos(cp), -math.acos(cp)):
                    if p > psi0 + 1e-13:
                        cands.append((p, zb))
        sd = (D - xc) / R
        pd = math.asin(sd) if abs(sd) <= 1.0 else math.inf
        if pd > psi0 and (not cands or pd <= min(cands)[0]):
            T += _arc_time(g, psi0, pd)
            L += R * (pd - psi0)
            return zc + sg * R * math.cos(pd), -sg * pd, T, L
        p1, zb = min(cands)
        T += _arc_time(g, psi0, p1)
        L += R * (p1 - psi0)
        x = xc + R * math.sin(p1)
        z = zb
        th = -sg * p1
        up = th > 0.0
    raise RuntimeError("ray did not reach the range")


def eigenrays(knots, p, s, n_fan: int = 2001, max_angle: float = 0.35):
    """Every ray from p that passes through s, found by shooting a fan of
    grazing angles in their vertical plane: list of (theta_p, T, L, theta_s)
    sorted by travel time."""
    prof = Profile(knots)
    p = np.asarray(p, float)
    s = np.asarray(s, float)
    D = math.hypot(*(s - p)[:2])
    ths = np.linspace(-max_angle, max_angle, n_fan)
    f = np.array([walk(prof, p[2], t, D)[0] - s[2] for t in ths])
    out = []
    for k in np.where(np.sign(f[:-1]) != np.sign(f[1:]))[0]:
        t = brentq(lambda a: walk(prof, p[2], a, D)[0] - s[2], ths[k], ths[k + 1], xtol=1e-15, rtol=1e-15)
        z, th, T, L = walk(prof, p[2], t, D)
        if abs(z - s[2]) < 1e-7:          # a root, not a jump across a shadow boundary
            out.append((t, T, L, th))
    return sorted(out, key=lambda r: r[1])
