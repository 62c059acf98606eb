// One ping of the volumetric sonar model, fused in a single kernel.
//
// Per lane (one ray): ray generation in FP64 (Sec. III grid, stratified
// jitter) -> for each bounce: FP32 nearest-hit traversal of the BVH with an
// LDS stack, along a straight line or, in a linear sound-speed gradient, along
// the exact circular arc that Snell's law gives (Sec. II-A) -> FP64
// re-intersection of the winner -> scattering, spreading, absorption and
// phase (Sec. II-B) -> for later bounces a connection (eigenray) to the sensor
// with an any-hit visibility query -> mirror continuation.
// Per wavefront: the rays of a beam sit in adjacent lanes (64 / N_r beams per
// wave); their contributions are reduced in a fixed order in LDS and each
// beam's whole range column is written once with coalesced stores, zeros
// included (a beam is the complex sum over its bundle of rays, Sec. II-B). No global
// atomics, no memset, bit-reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.hpp"

#include "trace.hpp"

namespace sonar {


// First hit of a ray: the triangle record, FP64 arc length along the whole
// path, one-way time, hit point, facet normal and arrival tangent.
struct Hit64 {
    bool ok;
    TriF tr;
    d3 nh, X, din;
    double s, tau;
};

// Piecewise-linear sound speed: the layer holding z (a point on a knot
// belongs to the layer above it).
__device__ __forceinline__ int layer_of(const PingArgs &a, double z)
{
    int i = 0;
    while (i + 1 < a.n_layers && z >= a.lay_z[i + 1]) ++i;
    return i;
}

// Arc length at which path p leaves layer i and the layer it enters (-1:
// never). Along a circle of curvature k the grazing angle is th0 - k s; at a
// boundary z_b Snell's invariant gives cos(th_b) = cos(th0) c(z_b) / c(o),
// reached going up at the upper boundary and going down at the lower one.
__device__ double layer_exit(const PingArgs &a, const int i, const Path64 &p, const double g, const double c0, int &next)
{
    double best = INFINITY;
    next = -1;
    const bool up = i + 1 < a.n_layers, down = i > 0;
    if (!p.arc) {
        if (p.d.z > 0.0 && up) {
            best = (a.lay_z[i + 1] - p.o.z) / p.d.z;
            next = i + 1;
        }
        if (p.d.z < 0.0 && down) {
            best = (a.lay_z[i] - p.o.z) / p.d.z;
            next = i - 1;
        }
        return best;
    }
    const double th0 = asin(fmin(1.0, fmax(-1.0, p.d.z)));
    const double cth = sqrt(p.d.x * p.d.x + p.d.y * p.d.y), co = c0 + g * p.o.z;
    for (int t = 0; t < 2; ++t) {
        if (t == 0 ? !up : !down) continue;
        const double zb = t == 0 ? a.lay_z[i + 1] : a.lay_z[i];
        const double C = cth * (c0 + g * zb) / co;
        if (C > 1.0) continue;
        const double thb = t == 0 ? acos(C) : -acos(C);
        const double s = (th0 - thb) / p.kappa;
        if (s > 1e-12 && s < best) {
            best = s;
            next = t == 0 ? i + 1 : i - 1;
        }
    }
    return best;
}

// First hit through the layers: each layer's circle is traversed as its own
// chord segment, in path order, until a hit inside the layer, the end of the
// time window or a layer the ray never leaves (`skip`: the facet the segment
// leaves from).
template <int DEPTH, int DL, bool STATS>
__device__ Hit64 first_hit_layered(const PingArgs &a, d3 o, d3 d, const double T_lim, const uint32_t skip,
                                   uint32_t *__restrict__ W, const int lane, bool &overflow, uint32_t &n_nodes,
                                   uint32_t &n_tris, uint32_t &n_deep)
{
    Hit64 h;
    h.ok = false;
    int layer = layer_of(a, o.z);
    if (layer > 0 && o.z == a.lay_z[layer] && d.z < 0.0) --layer;      // on a knot looking down
    double t_acc = 0.0, s_acc = 0.0;
    for (int piece = 0; piece < 64; ++piece) {
        const double g = a.lay_g[layer], c0 = a.lay_c0[layer];
        const Path64 path = make_path(o, d, g, c0);
        int next;
        const double s_exit = layer_exit(a, layer, path, g, c0, next);
        const double s_cap = a.c_hi * (T_lim - t_acc);
        const double s_end = fmin(s_exit, s_cap);
        const double s_min = piece == 0 ? EPS_SELF : 0.0;
        if (s_end > s_min) {
            const Seg32 seg = make_seg(path, s_min, s_end * (1.0 + 1e-6));
            float sf;
            const int ti = traverse<DEPTH, DL, false, true, STATS>(as_global(a.nodes), as_global(a.tris), seg, skip,
                                                                   W, lane, overflow, sf, a.max_steps, n_nodes, n_tris,
                                                                   n_deep);
            if (ti >= 0) {
                const TriF tr = load_tri(as_global(a.tris), (uint32_t)ti);
                d3 nh;
                const double s = refine64(tr, path, (double)sf, nh);
                // a hit past the boundary lies on the next layer's circle
                if (s > s_min && s <= s_exit) {
                    h.tau = t_acc + path_time(path, s, g, c0);
                    h.ok = h.tau <= T_lim;
                    h.tr = tr;
                    h.nh = nh;
                    h.s = s_acc + s;
                    h.X = path_point(path, s);
                    h.din = path_tangent(path, s);
                    return h;
                }
            }
        }
        if (next < 0 || s_exit >= s_cap) break;
        t_acc += path_time(path, s_exit, g, c0);
        s_acc += s_exit;
        o = path_point(path, s_exit);
        d = path_tangent(path, s_exit);
        d = d * (1.0 / norm3(d));
        layer = next;
    }
    return h;
}

// ---------------------------------------------------------------------------
// Return eigenrays through the layers. Along a ray Snell's invariant
// xi = cos(theta) / c is fixed; crossing one layer between depths za and zb
// without turning, with s = |sin theta| = sqrt(1 - xi^2 c^2), a ray advances
// horizontally by X = xi |dz| (ca + cb) / (sa + sb), travels arc length
// |asin sa - asin sb| / (xi |g|) and takes |atanh sa - atanh sb| / |g|; both
// are evaluated in forms free of cancellation (sin of the angle difference
// = xi g dz (ca + cb) / (sa cb + sb ca); the time as one log1p). A ray family
// has a reference depth zr: the turning depth (xi = 1 / c(zr)) or, for the
// direct ray, the depth of the span's largest speed (xi = (1 - u) / c(zr)).
// Walking away from zr the speed deficit e = c(zr) - c(z) is accumulated
// layer by layer from e(zr) = 0, so 1 - xi c(z) = (e + u c(z)) / c(zr) stays
// accurate next to a turning point.
struct LRun {
    double X, L, T;
    double e_lo, e_hi;      // speed deficits at the lower and upper end of the span
};

__device__ __forceinline__ double lay_speed(const PingArgs &a, double z)
{
    const int i = layer_of(a, z);
    return a.lay_c0[i] + a.lay_g[i] * z;
}

__device__ __forceinline__ double lay_sine(double e, double u, double c, double inv_cr)
{
    const double q = (e + u * c) * inv_cr;      // 1 - xi c
    return q > 0.0 ? sqrt(q * (2.0 - q)) : 0.0;
}

// Walk from z0 to z1 (either direction), each layer crossed once, adding to
// t; e is the speed deficit at z0 on entry and at z1 on return. FULL adds
// arc length and time to the horizontal run; `times` counts the walk twice
// (the two legs of a turning ray).
template <bool FULL>
__device__ __forceinline__ void lay_walk(const PingArgs &a, double cr, double u, double z0, double z1, double &e,
                                         double times, LRun &t)
{
    const double inv = 1.0 / cr, xi = (1.0 - u) * inv;
    const bool up = z1 >= z0;
    int i = layer_of(a, z0);
    if (!up && i > 0 && z0 == a.lay_z[i]) --i;          // going down from a knot: the layer below
    double z = z0;
    double ca = a.lay_c0[i] + a.lay_g[i] * z;
    double sa = lay_sine(e, u, ca, inv);
    for (int step = 0; step < MAX_SSP_KNOTS && z != z1; ++step) {
        const double edge = up ? (i + 1 < a.n_layers ? a.lay_z[i + 1] : INFINITY) : (i > 0 ? a.lay_z[i] : -INFINITY);
        const double zb = up ? fmin(edge, z1) : fmax(edge, z1);
        const double g = a.lay_g[i], dzs = zb - z, dz = fabs(dzs);
        const double cb = a.lay_c0[i] + g * zb;
        const double eb = e - g * dzs;
        const double sb = lay_sine(eb, u, cb, inv);
        if (sa + sb == 0.0) {
            // level at both ends: endless in a constant layer, else a rounding sliver
            if (g == 0.0) {
                t.X = t.L = t.T = INFINITY;
            } else if (FULL) {
                t.L += times * dz;
                t.T += times * dz / ca;
            }
        } else {
            t.X += times * (xi * dz * (ca + cb) / (sa + sb));
            if (FULL) {
                const double m = (ca + cb) / (sa * cb + sb * ca);
                const double y = fmin(1.0, xi * fabs(g) * dz * m);
                t.L += times * (dz * m * (y > 0.0 ? asin(y) / y : 1.0));
                const double q = (1.0 + m) / ((1.0 + sb) * ca);
                t.T += times * (g != 0.0 ? fabs(log1p(g * dzs * q) / g) : dz * q);
            }
        }
        z = zb;
        e = eb;
        ca = cb;
        sa = sb;
        i += up ? 1 : -1;
    }
}

// family 0: direct, reference zr = the span's fastest depth with u; 1 and 2:
// turning at zr above zhi or below zlo (u = 0)
template <bool FULL>
__device__ __forceinline__ LRun lay_family(const PingArgs &a, int fam, double zr, double u, double zlo, double zhi)
{
    LRun t{0.0, 0.0, 0.0, 0.0, 0.0};
    const double cr = lay_speed(a, zr);
    double e = 0.0;
    if (fam == 0) {
        lay_walk<FULL>(a, cr, u, zr, zlo, e, 1.0, t);
        t.e_lo = e;
        e = 0.0;
        lay_walk<FULL>(a, cr, u, zr, zhi, e, 1.0, t);
        t.e_hi = e;
    } else if (fam == 1) {
        lay_walk<FULL>(a, cr, 0.0, zr, zhi, e, 2.0, t);
        t.e_hi = e;
        lay_walk<FULL>(a, cr, 0.0, zhi, zlo, e, 1.0, t);
        t.e_lo = e;
    } else {
        lay_walk<FULL>(a, cr, 0.0, zr, zlo, e, 2.0, t);
        t.e_lo = e;
        lay_walk<FULL>(a, cr, 0.0, zlo, zhi, e, 1.0, t);
        t.e_hi = e;
    }
    return t;
}

// Root of f on [pa, pb] (f <= 0 at one end only) by the Illinois variant of
// regula falsi, to a relative bracket of 1e-15 or |f| <= 1e-15 d.
template <class F>
__device__ __forceinline__ double illinois(const F &f, double pa, double fa, double pb, double fb, double d)
{
    int side = 0;
    double pc = 0.5 * (pa + pb);
    for (int it = 0; it < 100; ++it) {
        pc = (pa * fb - pb * fa) / (fb - fa);
        if (!(pc > fmin(pa, pb) && pc < fmax(pa, pb))) pc = 0.5 * (pa + pb);
        if (pc == pa || pc == pb) break;
        const double fc = f(pc);
        if (fabs(fc) <= 1e-15 * d) break;
        if ((fc <= 0.0) == (fb <= 0.0)) {
            pb = pc;
            fb = fc;
            if (side == -1) fa *= 0.5;
            side = -1;
        } else {
            pa = pc;
            fa = fc;
            if (side == 1) fb *= 0.5;
            side = 1;
        }
        if (fabs(pb - pa) <= 1e-15 * fmax(fabs(pa), fabs(pb))) break;
    }
    return pc;
}

constexpr int EIG_CELLS = 64;      // turning-depth scan cells, uniform in sqrt(rise / window)

struct LConn {
    double L, T;
    d3 w, arrive;
    bool ok;
};

// The first-arriving eigenray with at most one turning point from P to S:
// the direct ray (its horizontal run shrinks as u = 1 - xi c_max grows;
// root in sqrt(u)), or a ray turning above the span or below it, at a depth
// where c exceeds every speed met on the way there. Turning depths within
// H = 2 r_max of the span are scanned at rises H (j / 64)^2 plus the ends of
// each turning interval; every sign change of the run's mismatch is refined
// in sqrt(rise / H). A family's scan ends once a lower bound of a turning
// ray's time passes the best arrival found. ok = false: no eigenray (an
// acoustic shadow).
__device__ __forceinline__ LConn connect_layered(const PingArgs &a, const d3 P, const d3 S)
{
    LConn c;
    c.ok = false;
    const d3 v = S - P;
    const double D = sqrt(v.x * v.x + v.y * v.y);
    const double zlo = fmin(P.z, S.z), zhi = fmax(P.z, S.z);
    double zm = lay_speed(a, zlo) >= lay_speed(a, zhi) ? zlo : zhi;
    for (int i = 1; i < a.n_layers; ++i) {
        const double zk = a.lay_z[i];
        if (zk > zlo && zk < zhi && a.lay_c0[i] + a.lay_g[i] * zk > lay_speed(a, zm)) zm = zk;
    }
    const double cm = lay_speed(a, zm);
    int best_fam = -1;
    double best_zr = 0.0, best_u = 0.0;
    LRun best{0.0, INFINITY, INFINITY, 0.0, 0.0};
    // direct family
    if (zlo == zhi) {
        if (a.lay_g[layer_of(a, zlo)] == 0.0 && D > 0.0) {
            best_fam = 0;
            best_zr = zm;
            best = LRun{D, D, D / cm, 0.0, 0.0};          // level in a constant layer
        }
    } else if (D == 0.0) {
        best_fam = 0;
        best_zr = zm;
        best_u = 1.0;
        best = lay_family<true>(a, 0, zm, 1.0, zlo, zhi);
    } else {
        auto f = [&](double w) { return lay_family<false>(a, 0, zm, w * w, zlo, zhi).X - D; };
        const double f0 = f(0.0);
        if (f0 > 0.0) {
            const double w = illinois(f, 0.0, f0, 1.0, -D, D);
            best_fam = 0;
            best_zr = zm;
            best_u = w * w;
            best = lay_family<true>(a, 0, zm, best_u, zlo, zhi);
        }
    }
    // turning families
    const double H = 2.0 * a.r_max, span = zhi - zlo;
    for (int fam = 1; fam <= 2; ++fam) {
        const double dir = fam == 1 ? 1.0 : -1.0, z0 = fam == 1 ? zhi : zlo, zend = z0 + dir * H;
        auto zt_of = [&](double vv) { return z0 + dir * (H * (vv * vv)); };
        auto f = [&](double vv) { return lay_family<false>(a, fam, zt_of(vv), 0.0, zlo, zhi).X - D; };
        // A ray turning at rise r travels at least sqrt(D^2 + (2 r + span)^2)
        // at no more than the window's largest speed: once that bound passes
        // the best arrival, no later turning depth can arrive first.
        double c_win = fmax(lay_speed(a, z0), lay_speed(a, zend));
        for (int k = 1; k < a.n_layers; ++k)
            if (dir * (a.lay_z[k] - z0) > 0.0 && dir * (zend - a.lay_z[k]) > 0.0)
                c_win = fmax(c_win, a.lay_c0[k] + a.lay_g[k] * a.lay_z[k]);
        auto slower = [&](double vv) {
            const double vert = 2.0 * H * (vv * vv) + span;
            return sqrt(D * D + vert * vert) >= best.T * c_win;
        };
        double M = cm, z = z0;
        int i = layer_of(a, z0);
        if (fam == 2 && i > 0 && z0 == a.lay_z[i]) --i;
        bool done = false;
        for (int step = 0; step < MAX_SSP_KNOTS && !done && i >= 0 && i < a.n_layers; ++step) {
            const double g = a.lay_g[i], c0 = a.lay_c0[i];
            const double edge = fam == 1 ? (i + 1 < a.n_layers ? a.lay_z[i + 1] : INFINITY)
                                         : (i > 0 ? a.lay_z[i] : -INFINITY);
            const double zb = fam == 1 ? fmin(edge, zend) : fmax(edge, zend);
            if (g * dir > 0.0) {
                // turning interval of this layer: from where c passes the record M to zb
                const double zs = (M - c0) / g;
                const double ta = fam == 1 ? fmax(zs, z) : fmin(zs, z);
                if (dir * (zb - ta) > 0.0) {
                    const double va = sqrt(fabs(ta - z0) / H), vb = sqrt(fabs(zb - z0) / H);
                    if (slower(va)) {
                        done = true;
                        break;
                    }
                    double vp = va, fp = f(va);
                    for (int j = (int)floor(va * EIG_CELLS) + 1;; ++j) {
                        double vq = (double)j / EIG_CELLS;
                        const bool last = vq >= vb;
                        if (last) vq = vb;
                        if (vq <= vp) continue;
                        if (slower(vp)) {
                            done = true;
                            break;
                        }
                        const double fq = f(vq);
                        if ((fq <= 0.0) != (fp <= 0.0)) {
                            const double vr = illinois(f, vp, fp, vq, fq, D);
                            const double zr = zt_of(vr);
                            const LRun r = lay_family<true>(a, fam, zr, 0.0, zlo, zhi);
                            if (r.T < best.T) {
                                best = r;
                                best_fam = fam;
                                best_zr = zr;
                                best_u = 0.0;
                            }
                        }
                        if (last) break;
                        vp = vq;
                        fp = fq;
                    }
                }
                M = fmax(M, c0 + g * zb);
            }
            if (dir * (zb - zend) >= 0.0) break;
            z = zb;
            i += fam == 1 ? 1 : -1;
        }
    }
    if (best_fam < 0) return c;
    c.ok = true;
    c.L = best.L;
    c.T = best.T;
    const double cr = lay_speed(a, best_zr), xi = (1.0 - best_u) / cr;
    const double ux = D > 0.0 ? v.x / D : 0.0, uy = D > 0.0 ? v.y / D : 0.0;
    const double cP = lay_speed(a, P.z), cS = lay_speed(a, S.z);
    const bool p_low = P.z <= S.z;
    const double sp = lay_sine(p_low ? best.e_lo : best.e_hi, best_u, cP, 1.0 / cr);
    const double ss = lay_sine(p_low ? best.e_hi : best.e_lo, best_u, cS, 1.0 / cr);
    const double upd = S.z > P.z ? 1.0 : (S.z < P.z ? -1.0 : 0.0);
    const double vp = best_fam == 0 ? upd : (best_fam == 1 ? 1.0 : -1.0);
    const double vs = best_fam == 0 ? upd : (best_fam == 1 ? -1.0 : 1.0);
    const d3 w = mk3(xi * cP * ux, xi * cP * uy, vp * sp), ar = mk3(xi * cS * ux, xi * cS * uy, vs * ss);
    c.w = w * (1.0 / norm3(w));
    c.arrive = ar * (1.0 / norm3(ar));
    return c;
}

// Occlusion of a layered return path leaving P along w for arc length L:
// one circle per layer, each piece an any-hit query over its part of
// (EPS_SELF, L - EPS_SELF), the facet `skip` excluded.
template <int DEPTH, int DL, bool STATS>
__device__ __forceinline__ bool occluded_layered(const PingArgs &a, const d3 P, const d3 w, const double L, const uint32_t skip,
                                 uint32_t *__restrict__ W, const int lane, bool &overflow, uint32_t &n_nodes,
                                 uint32_t &n_tris, uint32_t &n_deep)
{
    int layer = layer_of(a, P.z);
    if (layer > 0 && P.z == a.lay_z[layer] && w.z < 0.0) --layer;
    d3 o = P, d = w;
    double s0 = 0.0;
    for (int piece = 0; piece < 64; ++piece) {
        const double g = a.lay_g[layer], c0 = a.lay_c0[layer];
        const Path64 path = make_path(o, d, g, c0);
        int next;
        const double s_exit = layer_exit(a, layer, path, g, c0, next);
        const double lo = fmax(EPS_SELF - s0, 0.0), hi = fmin(s_exit, L - EPS_SELF - s0);
        if (hi > lo) {
            const Seg32 seg = make_seg(path, lo, hi);
            float sf;
            const int hb = traverse<DEPTH, DL, true, true, STATS>(as_global(a.nodes), as_global(a.tris), seg, skip, W,
                                                                  lane, overflow, sf, a.max_steps, n_nodes, n_tris,
                                                                  n_deep);
            if (hb >= 0) return true;
        }
        if (next < 0 || s0 + s_exit >= L) break;
        s0 += s_exit;
        o = path_point(path, s_exit);
        d = path_tangent(path, s_exit);
        d = d * (1.0 / norm3(d));
        layer = next;
    }
    return false;
}


// The ping body for one block of consecutive rays (blockDim.x of them, one
// lane each, starting at ray0; a multiple of 64). `a` is the ping's argument
// block (kernel arguments, or a batch descriptor in device memory); `W` is
// this wavefront's LDS area.
template <int DEPTH, int K, bool ARC, bool STATS, bool LAYERED = false, bool RETRO = false>
__device__ __forceinline__ void ping_tile(const PingArgs &a, const int64_t ray0, uint32_t *__restrict__ W)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    const int64_t gid = ray0 + threadIdx.x;
    const int64_t beam = gid >> a.log2_nr;
    const int j = (int)(gid & (a.n_r - 1));
    const bool active = beam < a.n_beams;

    // Contribution slots: registers for a single bounce; for several bounces
    // an LDS area past the traversal stack, slot (k, lane) at k * 64 + lane,
    // with the retro-chain returns of vertices 1..K-1 in slots K..2K-2.
    constexpr int KS = RETRO ? 2 * K - 1 : K;
    constexpr int DLS = K == 1 ? K1_LDS_STACK : (RETRO ? kn_lds_stack_retro(K) : KN_LDS_STACK);
    constexpr int DL = DEPTH > DLS ? DLS : DEPTH;
    int *sbin = (K == 1) ? reinterpret_cast<int *>(W) : reinterpret_cast<int *>(W + DL * WAVE);
    float4 *sval = (K == 1) ? reinterpret_cast<float4 *>(W + K1_BIN_WORDS)
                            : reinterpret_cast<float4 *>(W + DL * WAVE + KS * WAVE);
    Slot slot0 = Slot{-1, 0.f, 0.f, 0.f};
    if (K > 1) {
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            sbin[k * WAVE + lane] = -1;
            sval[k * WAVE + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    float gfeat[7] = {0, 0, 0, 0, 0, 0, 0};
    bool overflow = false;
    uint32_t st_nodes = 0, st_tris = 0, st_deep = 0;     // traversal work of this ray

    if (active) {
        // ---- ray generation (FP64)
        const int h = (int)(beam % a.beams_h), v = (int)(beam / a.beams_h);
        double az, el;
        float w_tx = 1.f;            // transmit pattern at the launch direction
        if (a.grid_mode == 1) {
            az = -0.5 * a.hfov + h * a.dth_h;
            el = -0.5 * a.vfov + v * a.dth_v;
        } else {
            const int ja = j % a.na, je = j / a.na;
            double u1 = 0.5, u2 = 0.5;
            if (a.jitter) {
                uint64_t ctr = ((uint64_t)a.ping << 40) ^ ((uint64_t)beam << 8) ^ (uint64_t)j;
                uint64_t z = splitmix64_nth(a.seed, ctr + 1);
                u1 = (double)(z >> 40) * (1.0 / 16777216.0);
                u2 = (double)((z >> 16) & 0xFFFFFFu) * (1.0 / 16777216.0);
            }
            az = -0.5 * a.hfov + (h + (ja + u1) / a.na) * a.dth_h;
            el = -0.5 * a.vfov + (v + (je + u2) / a.ne) * a.dth_v;
            if (a.flags & FLAG_BEAM_PATTERN) {
                // offsets from the beam centre in cells: lobe = 2^(-2 (fa^2 + fe^2))
                const float fa = (float)((ja + u1) / a.na - 0.5), fe = (float)((je + u2) / a.ne - 0.5);
                w_tx = exp2f(-2.f * (fa * fa + fe * fe));
            }
        }
        double ce = cos(el), se = sin(el), ca = cos(az), sa = sin(az);
        d3 ds = mk3(ce * ca, ce * sa, se);
        d3 d = mk3(a.rot[0] * ds.x + a.rot[1] * ds.y + a.rot[2] * ds.z,
                   a.rot[3] * ds.x + a.rot[4] * ds.y + a.rot[5] * ds.z,
                   a.rot[6] * ds.x + a.rot[7] * ds.y + a.rot[8] * ds.z);
        const d3 S = mk3(a.pos[0], a.pos[1], a.pos[2]);
        d3 o = S;
        double L_out = 0.0, T_out = 0.0, Wt = 1.0;
        uint32_t prev = 0xFFFFFFFFu;
        const size_t ray = (size_t)gid;
        const bool masked = a.mask && ((a.mask[ray >> 5] >> (ray & 31)) & 1u);
        bool stop = false;

#pragma unroll
        for (int k = 0; k < K; ++k) {
            int rec_tri = -1, rec_vis = 0;
            int cbin = -1;
            float cre = 0.f, cim = 0.f, cinc = 0.f;
            float w_rx = w_tx;       // receive pattern: bounce 1 arrives along the launch ray
            int rxb = (int)beam;     // the beam the return is added to
            int rbin = -1;           // retro-chain return of this vertex
            float rre = 0.f, rim = 0.f, rinc = 0.f;
            if (!stop) {
                // segment limit: arc length for constant c, travel time in a gradient
                double s_lim, T_lim = 0.0;
                if (!ARC) {
                    s_lim = (K == 1) ? a.r_max : 2.0 * a.r_max - L_out;
                } else {
                    T_lim = (K == 1) ? a.r_max / a.c_ref : 2.0 * a.r_max / a.c_ref - T_out;
                    s_lim = a.c_hi * T_lim;
                }
                stop = true;
                if (s_lim > EPS_SELF) {
                    Hit64 hit;
                    Path64 path;
                    float sf = 0.f;
                    int ti;
                    if constexpr (LAYERED) {
                        hit = first_hit_layered<DEPTH, DL, STATS>(a, o, d, T_lim, prev, W, lane, overflow, st_nodes,
                                                                  st_tris, st_deep);
                        ti = hit.ok ? 0 : -1;
                    } else {
                        path = ARC ? make_path(o, d, a.g, a.c0) : Path64{o, d, mk3(0, 0, 0), 0.0, false};
                        const Seg32 seg = make_seg(path, EPS_SELF, s_lim * (1.0 + 1e-6));
                        // in a gradient a vertical ray is a degenerate arc (kappa = 0)
                        ti = traverse<DEPTH, DL, false, ARC, STATS>(as_global(a.nodes), as_global(a.tris), seg, prev, W,
                                                                    lane, overflow, sf, a.max_steps, st_nodes, st_tris,
                                                                    st_deep);
                    }
                    if (ti >= 0) {
                        TriF tr;
                        d3 nh;
                        double s, tau;
                        bool ok;
                        if constexpr (LAYERED) {
                            tr = hit.tr;
                            nh = hit.nh;
                            s = hit.s;
                            tau = hit.tau;
                            ok = true;
                        } else {
                            tr = load_tri(as_global(a.tris), (uint32_t)ti);
                            s = refine64(tr, path, (double)sf, nh);
                            tau = ARC ? path_time(path, s, a.g, a.c0) : s / a.c0;
                            ok = s > EPS_SELF && (ARC ? tau <= T_lim : s <= s_lim);
                        }
                        if (ok) {
                            stop = false;
                            uint32_t id = tr.idbits & 0x7FFFFFFFu;
                            rec_tri = (int)id;
                            d3 X, din;
                            if constexpr (LAYERED) {
                                X = hit.X;
                                din = hit.din;
                            } else {
                                X = ARC ? path_point(path, s) : o + d * s;
                                din = ARC ? path_tangent(path, s) : d;
                            }
                            L_out += s;
                            T_out += tau;
                            double dn = dot3(nh, din);
                            d3 np = dn > 0.0 ? nh * -1.0 : nh;
                            double cos_i = -dot3(np, din);
                            d3 rh = din - np * (2.0 * dot3(np, din));
                            const bool pr = (tr.idbits & MAT_BIT) != 0;
                            double rho = pr ? 1.0 : (double)tr.rho;
                            double kd = pr ? 0.0 : a.k_d;
                            double ks = pr ? 1.0 : a.k_s;
                            double phi = pr ? 0.0 : (double)tr.phi;
                            double sgn = pr ? -1.0 : 1.0;

                            // Return path and contribution first, visibility last: only the
                            // contribution and the continuation state stay live across the
                            // any-hit traversal.
                            double L_back, T_back;
                            d3 w;
                            bool vis = true;
                            if (k == 0) {
                                L_back = L_out;
                                T_back = T_out;
                                w = din * -1.0;
                            } else {
                                Conn cn;
                                if constexpr (LAYERED) {
                                    const LConn lc = connect_layered(a, X, S);
                                    cn = Conn{lc.L, lc.T, lc.w, lc.arrive};
                                    if (!lc.ok) {
                                        // no eigenray reaches the sensor: a shadow zone
                                        vis = false;
                                        cn = Conn{0.0, 0.0, mk3(0.0, 0.0, 0.0), mk3(0.0, 0.0, 0.0)};
                                    }
                                } else {
                                    cn = connect(X, S, ARC ? a.g : 0.0, a.c0);
                                }
                                L_back = cn.L;
                                T_back = cn.T;
                                w = cn.w;
                                // arrival direction (from S toward P) inside the field of view
                                const d3 av = cn.arrive * -1.0;
                                const double sx = a.rot[0] * av.x + a.rot[3] * av.y + a.rot[6] * av.z;
                                const double sy = a.rot[1] * av.x + a.rot[4] * av.y + a.rot[7] * av.z;
                                const double sz = a.rot[2] * av.x + a.rot[5] * av.y + a.rot[8] * av.z;
                                const double sxy = sqrt(sx * sx + sy * sy);
                                if (a.hfov < M_PI) {
                                    // |az| <= hfov / 2 and |el| <= vfov / 2 without inverse trigonometry
                                    if (!(sx > 0.0 && fabs(sy) <= a.tan_h * sx)) vis = false;
                                } else if (fabs(atan2(sy, sx)) > 0.5 * a.hfov) {
                                    vis = false;
                                }
                                if (fabs(sz) > a.tan_v * sxy) vis = false;
                                if (vis && a.flags) {
                                    // receive cell and pattern at the arrival direction
                                    const double xa = (atan2(sy, sx) + 0.5 * a.hfov) / a.dth_h;
                                    const double xe = (atan2(sz, sxy) + 0.5 * a.vfov) / a.dth_v;
                                    int hr = h, vr = v;
                                    if (a.flags & FLAG_RX_BEAMS) {
                                        hr = min(max((int)floor(xa), 0), a.beams_h - 1);
                                        vr = min(max((int)floor(xe), 0), a.beams_v - 1);
                                        rxb = vr * a.beams_h + hr;
                                    }
                                    if (a.flags & FLAG_BEAM_PATTERN) {
                                        const float fa = (float)(xa - (hr + 0.5)), fe = (float)(xe - (vr + 0.5));
                                        w_rx = exp2f(-2.f * (fa * fa + fe * fe));
                                    }
                                }
                            }
                            double cos_o = dot3(np, w);
                            if (vis && cos_o > 0.0) {
                                const double Tt = T_out + T_back;
                                const double reff = a.c_ref * Tt / 2.0;
                                const double fb = floor((reff - a.r_min) / a.dr);
                                if (fb >= 0.0 && fb < (double)a.n_bins) {
                                    float lobe = (float)dot3(rh, w);
                                    lobe = lobe > 0.f ? lobe : 0.f;
                                    const double spec = ks != 0.0 ? ks * (double)powf(lobe, (float)a.phong_n) : 0.0;
                                    const double fsc = rho * (kd * cos_i * cos_o + spec);
                                    const double att =
                                        (double)expf((float)(-a.alpha_db * (L_out + L_back) * LN10_OVER_20));
                                    const double amp = Wt * sgn * sqrt(fsc) * att / (L_out * L_back * a.n_r);
                                    const double cyc = a.f0 * Tt;
                                    double ph = TWO_PI * (cyc - floor(cyc)) + phi;
                                    ph -= TWO_PI * rint(ph / TWO_PI);
                                    float sn, cs;
                                    sincosf((float)ph, &sn, &cs);
                                    cbin = (int)fb;
                                    cre = (float)amp * cs;
                                    cim = (float)amp * sn;
                                    cinc = (float)(amp * amp);
                                    if (k == 0) {
                                        gfeat[0] = (float)(reff / a.r_max);
                                        gfeat[1] = (float)cos_i;
                                        gfeat[2] = (float)rho;
                                        gfeat[3] = (float)np.x;
                                        gfeat[4] = (float)np.y;
                                        gfeat[5] = (float)np.z;
                                        gfeat[6] = 1.f;
                                    }
                                }
                            }
                            if constexpr (RETRO) {
                                // back into the reversed incident direction and along the
                                // outgoing chain reversed: twice its time and length, its
                                // weight squared
                                if (k > 0) {
                                    float lobe = (float)(-dot3(rh, din));
                                    lobe = lobe > 0.f ? lobe : 0.f;
                                    const double spec = ks != 0.0 ? ks * (double)powf(lobe, (float)a.phong_n) : 0.0;
                                    const double fsc = rho * (kd * cos_i * cos_i + spec);
                                    const double fb = floor((a.c_ref * T_out - a.r_min) / a.dr);
                                    if (fb >= 0.0 && fb < (double)a.n_bins) {
                                        const double att =
                                            (double)expf((float)(-a.alpha_db * 2.0 * L_out * LN10_OVER_20));
                                        const double amp = Wt * Wt * sgn * sqrt(fsc) * att / (L_out * L_out * a.n_r);
                                        const double cyc = a.f0 * 2.0 * T_out;
                                        double ph = TWO_PI * (cyc - floor(cyc)) + phi;
                                        ph -= TWO_PI * rint(ph / TWO_PI);
                                        float sn, cs;
                                        sincosf((float)ph, &sn, &cs);
                                        rbin = (int)fb;
                                        rre = (float)amp * cs;
                                        rim = (float)amp * sn;
                                        rinc = (float)(amp * amp);
                                    }
                                }
                            }
                            // continuation along the mirror direction, or drawn from the lobes
                            if (k + 1 < K) {
                                d3 dc = rh;
                                if ((a.flags & FLAG_DIFFUSE_BOUNCE) && !pr) {
                                    Wt *= sqrt(rho * (kd + ks)) * sgn;
                                    if (Wt != 0.0) {
                                        const Drawn dw = draw_continuation(a.seed, a.ping, a.phong_n, ray, k, rh, np,
                                                                           kd, ks);
                                        if (!dw.lit) Wt = 0.0;
                                        dc = dw.dir;
                                    }
                                } else {
                                    Wt *= sqrt(rho * ks) * sgn;
                                }
                                const double dS = norm3(X - S);
                                const double lb = ARC ? a.c_ref * (T_out + dS / a.c_hi) / 2.0 : (L_out + dS) / 2.0;
                                if (Wt == 0.0 || lb >= a.r_max) stop = true;
                                o = X;
                                d = dc;
                                prev = id;
                            }
                            // visibility of the connection: any hit other than this facet
                            if (k > 0 && vis && L_back > 2.0 * EPS_SELF) {
                                bool blocked;
                                if constexpr (LAYERED) {
                                    blocked = occluded_layered<DEPTH, DL, STATS>(a, X, w, L_back, id, W, lane, overflow,
                                                                                 st_nodes, st_tris, st_deep);
                                } else {
                                    const Path64 cp =
                                        ARC ? make_path(X, w, a.g, a.c0) : Path64{X, w, mk3(0, 0, 0), 0.0, false};
                                    const Seg32 cs = make_seg(cp, EPS_SELF, L_back - EPS_SELF);
                                    float sa2;
                                    blocked = traverse<DEPTH, DL, true, ARC, STATS>(as_global(a.nodes), as_global(a.tris),
                                                                                   cs, id, W, lane, overflow, sa2,
                                                                                   a.max_steps, st_nodes, st_tris,
                                                                                   st_deep) >= 0;
                                }
                                if (blocked) {
                                    vis = false;
                                    cbin = -1;
                                    cre = cim = cinc = 0.f;
                                }
                            }
                            rec_vis = vis ? 1 : 0;
                        }
                    }
                }
            }
            if (a.flags & FLAG_BEAM_PATTERN) {
                const float wgt = w_tx * w_rx;
                cre *= wgt;
                cim *= wgt;
                cinc *= wgt * wgt;
                if constexpr (RETRO) {
                    const float wr = w_tx * w_tx;      // out and back along the launch ray
                    rre *= wr;
                    rim *= wr;
                    rinc *= wr * wr;
                }
            }
            int cbin_here = cbin;    // the bin this lane's launch beam receives
            if (K > 1 && k > 0 && (a.flags & FLAG_RX_BEAMS)) {
                const bool away = cbin >= 0 && rxb != (int)beam;
                if (away) cbin_here = -1;
                rx_append(a, away && !masked, make_int4(rxb, cbin, __float_as_int(cre), __float_as_int(cim)), lane);
            }
            if (a.rec_tri) {
                size_t ri = ray * K + k;
                a.rec_tri[ri] = rec_tri;
                a.rec_bin[ri] = cbin;
                a.rec_vis[ri] = rec_vis;
                a.rec_amp[ri] = make_float2(cre, cim);
                if (a.rec_beam) a.rec_beam[ri] = rxb;
                if constexpr (RETRO) {
                    if (a.rec_rbin) {
                        a.rec_rbin[ri] = rbin;
                        a.rec_ramp[ri] = make_float2(rre, rim);
                    }
                }
            }
            if (K == 1) {
                slot0 = Slot{cbin_here, cre, cim, cinc};
            } else {
                sbin[k * WAVE + lane] = cbin_here;
                sval[k * WAVE + lane] = k == 0 ? make_float4(cre, cim, cinc, 0.f) : make_float4(cre, cim, 0.f, cinc);
                if constexpr (RETRO) {
                    if (k > 0) {
                        sbin[(K + k - 1) * WAVE + lane] = rbin;
                        sval[(K + k - 1) * WAVE + lane] = make_float4(rre, rim, 0.f, rinc);
                    }
                }
            }
        }
        if (STATS) {
            a.stats[3 * ray] = st_nodes;
            a.stats[3 * ray + 1] = st_tris;
            a.stats[3 * ray + 2] = st_deep;
        }
        if (masked) {
            slot0.bin = -1;
            if (K > 1) {
#pragma unroll
                for (int k = 0; k < KS; ++k) sbin[k * WAVE + lane] = -1;
            }
            for (int q = 0; q < 7; ++q) gfeat[q] = 0.f;
        }
    }
    if (overflow) atomicOr(a.status, ST_STACK);

    // ---- G-buffer: reduce the first-bounce features over the beam's lanes
    if (a.gbuf) {
        for (int off = 1; off < a.n_r; off <<= 1)
            for (int q = 0; q < 7; ++q) gfeat[q] += __shfl_xor(gfeat[q], off);
        if (active && j == 0) {
            float cnt = gfeat[6];
            float inv = cnt > 0.f ? 1.f / cnt : 0.f;
            // the beam axis (cell centre, or the grid node) in the world frame: its vertical component
            const int bh = (int)(beam % a.beams_h), bv = (int)(beam / a.beams_h);
            const float off = a.grid_mode == 1 ? 0.f : 0.5f;
            const float az = (float)(-0.5 * a.hfov) + ((float)bh + off) * (float)a.dth_h;
            const float el = (float)(-0.5 * a.vfov) + ((float)bv + off) * (float)a.dth_v;
            float sa, ca, se, ce;
            sincosf(az, &sa, &ca);
            sincosf(el, &se, &ce);
            const float up = (float)a.rot[6] * (ce * ca) + (float)a.rot[7] * (ce * sa) + (float)a.rot[8] * se;
            float4 *g = reinterpret_cast<float4 *>(a.gbuf + (size_t)beam * 8);
            g[0] = make_float4(gfeat[0] * inv, gfeat[1] * inv, gfeat[2] * inv, gfeat[3] * inv);
            g[1] = make_float4(gfeat[4] * inv, gfeat[5] * inv, cnt / a.n_r, up);
        }
    }

    // ---- accumulation: fixed-order reduction of equal (beam, bin) slots
    wave_sync();
    // column index: past the slots for one bounce, in the (now free) stack area otherwise
    uint32_t *sidx32 = (K == 1) ? W + K1_IDX_BASE : W;
    if (K == 1) {
        sbin[lane] = slot0.bin;
        sval[lane] = make_float4(slot0.re, slot0.im, slot0.inc, 0.f);
    }
    wave_sync();
    reduce_tile<KS>(a, ray0, wave, lane, j, active, sbin, sval, sidx32);
}

// STATS instantiations count traversal work per ray (a diagnostic: the
// counters cost registers, so the plain instantiations carry none).
// Occupancy targets: eight waves per SIMD for single-bounce straight rays
// (64 registers), three with several bounces.
template <int K, bool ARC>
constexpr int ping_waves_per_eu() { return K == 1 ? (ARC ? 5 : 8) : 3; }

template <int DEPTH, int K, bool ARC, bool STATS, bool LAYERED = false, bool RETRO = false>
__global__ __attribute__((amdgpu_flat_work_group_size(1, BLOCK), amdgpu_waves_per_eu(ping_waves_per_eu<K, ARC>())))
void k_ping(PingArgs a, int wave_words)
{
    extern __shared__ uint32_t lds[];
    uint32_t *W = lds + (size_t)(threadIdx.x / WAVE) * wave_words;
    if constexpr (LAYERED) {
        // The profile tables are indexed by layer at run time: read the
        // argument block where it lies (kernel-argument memory, the block is
        // the first argument), not from a private per-lane copy of it.
        const PingArgs *ka = (const PingArgs *)__builtin_amdgcn_kernarg_segment_ptr();
        ping_tile<DEPTH, K, ARC, STATS, LAYERED, RETRO>(*ka, (int64_t)xcd_remap(blockIdx.x, gridDim.x) * BLOCK, W);
    } else {
        ping_tile<DEPTH, K, ARC, STATS, LAYERED, RETRO>(a, (int64_t)xcd_remap(blockIdx.x, gridDim.x) * BLOCK, W);
    }
}

// Persistent batch: every block (WPB waves) pops items of `tiles_per_item`
// units from one device counter until the queue is empty; a unit is WPB * 64
// consecutive rays of one ping (a ping's rays are laid out in 256-ray tiles,
// so a unit never straddles two pings). Per-ping first-start and
// last-finish stamps come from the constant-rate device clock. All pings of
// a batch share the hierarchy depth class, bounce count and medium type
// (template arguments); layouts, rays per beam, poses and outputs come per
// ping from its descriptor.
template <int DEPTH, int K, bool ARC, bool LAYERED = false, bool RETRO = false, int WPB = WAVES_PER_BLOCK>
__global__ __attribute__((amdgpu_flat_work_group_size(1, BLOCK), amdgpu_waves_per_eu(ping_waves_per_eu<K, ARC>())))
void k_ping_batch(const PingArgs *__restrict__ desc, int n_pings,
                                                      uint32_t *__restrict__ queue, unsigned long long *__restrict__ t0,
                                                      unsigned long long *__restrict__ t1, int wave_words,
                                                      int tiles_per_item)
{
    extern __shared__ uint32_t lds[];
    __shared__ int s_item;
    constexpr int UNITS_PER_TILE = WAVES_PER_BLOCK / WPB;     // units in a 256-ray tile
    uint32_t *W = lds + (size_t)(threadIdx.x / WAVE) * wave_words;
    const PingArgs &last = desc[n_pings - 1];
    const int total_units = (last.tile_offset + last.n_tiles) * UNITS_PER_TILE;
    const int n_items = (total_units + tiles_per_item - 1) / tiles_per_item;
    while (true) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);     // uniform: descriptor fields in SGPRs
        __syncthreads();
        if (item >= n_items) break;
        for (int q = 0; q < tiles_per_item; ++q) {
            const int gu = item * tiles_per_item + q;
            if (gu >= total_units) break;
            const int gt = gu / UNITS_PER_TILE;
            // the ping holding global tile gt: last descriptor with tile_offset <= gt
            int lo = 0, hi = n_pings - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (desc[mid].tile_offset <= gt) lo = mid;
                else hi = mid - 1;
            }
            const PingArgs &a = desc[lo];
            const int64_t ray0 = (int64_t)(gu - a.tile_offset * UNITS_PER_TILE) * (WPB * WAVE);
            unsigned long long start = __builtin_amdgcn_s_memrealtime();
            if (ray0 < a.n_rays) ping_tile<DEPTH, K, ARC, false, LAYERED, RETRO>(a, ray0, W);
            __syncthreads();
            if (threadIdx.x == 0) {
                unsigned long long end = __builtin_amdgcn_s_memrealtime();
                atomicMin(&t0[lo], start);
                atomicMax(&t1[lo], end);
            }
        }
    }
}

// Resets the batch queue and the per-ping stamps (a kernel, not a memset, so
// that graph replays always start from the same state).
__global__ void k_batch_reset(uint32_t *queue, unsigned long long *t0, unsigned long long *t1, int n_pings)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *queue = 0u;
    if (i < n_pings) {
        t0[i] = ~0ull;
        t1[i] = 0ull;
    }
}

__global__ void k_rx_reset(uint32_t *count)
{
    if (threadIdx.x == 0) *count = 0u;
}

// Listed returns into their receive beams' columns (and the bounce >= 2
// incoherent channel); grid-stride over the list.
__global__ __launch_bounds__(256) void k_rx_scatter(const int4 *__restrict__ list, const uint32_t *__restrict__ count,
                                                    uint32_t cap, float2 *__restrict__ volume, float *__restrict__ incoh,
                                                    int n_bins, int64_t n_beams)
{
    const uint32_t n = min(*count, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int4 e = list[i];
        const size_t cell = (size_t)e.x * n_bins + e.y;
        const float re = __int_as_float(e.z), im = __int_as_float(e.w);
        atomicAdd(&volume[cell].x, re);
        atomicAdd(&volume[cell].y, im);
        if (incoh) atomicAdd(&incoh[(size_t)n_beams * n_bins + cell], re * re + im * im);
    }
}

// Receive binning in a batch: before the pings every list's counter is
// cleared, after them every ping's list is added into its volume (grid y
// strides over the pings; pings without a list are skipped at once).
__global__ void k_rx_reset_batch(const PingArgs *__restrict__ desc, int n_pings)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pings && desc[i].rx_count) *desc[i].rx_count = 0u;
}

__global__ __launch_bounds__(256) void k_rx_scatter_batch(const PingArgs *__restrict__ desc, int n_pings)
{
    for (int p = blockIdx.y; p < n_pings; p += gridDim.y) {
        const PingArgs &a = desc[p];
        if (!a.rx_list) continue;
        const uint32_t n = min(*a.rx_count, a.rx_cap);
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            const int4 e = a.rx_list[i];
            const size_t cell = (size_t)e.x * a.n_bins + e.y;
            const float re = __int_as_float(e.z), im = __int_as_float(e.w);
            atomicAdd(&a.volume[cell].x, re);
            atomicAdd(&a.volume[cell].y, im);
            if (a.incoh) atomicAdd(&a.incoh[(size_t)a.n_beams * a.n_bins + cell], re * re + im * im);
        }
    }
}

hipError_t launch_rx_reset(uint32_t *count, hipStream_t s)
{
    hipLaunchKernelGGL(k_rx_reset, dim3(1), dim3(64), 0, s, count);
    return hipGetLastError();
}

hipError_t launch_rx_scatter(const PingArgs &a, hipStream_t s)
{
    // at most rx_cap entries, grid-stride over up to 2,048 blocks
    const uint64_t want = ((uint64_t)a.rx_cap + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 2048 ? want : 2048);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rx_scatter, dim3(blocks), dim3(256), 0, s, a.rx_list, a.rx_count, a.rx_cap, a.volume,
                       a.incoh, a.n_bins, (int64_t)a.n_beams);
    return hipGetLastError();
}

int ping_wave_words(int depth, int n_bins, int K, bool retro = false)
{
    if (K > 1) {   // LDS stack + slots; the column index reuses the stack
        const int dls = retro ? kn_lds_stack_retro(K) : KN_LDS_STACK;
        return (depth > dls ? dls : depth) * WAVE + 5 * WAVE * (retro ? 2 * K - 1 : K);
    }
    const int stk = (depth > K1_LDS_STACK ? K1_LDS_STACK : depth) * WAVE;
    const int acc = K1_IDX_BASE + (n_bins + 1) / 2;
    const int w = acc > stk ? acc : stk;
    return (w + 3) & ~3;                              // keeps every wave's float4 slots 16-byte aligned
}

// Retro-chain returns take their own instantiations (deep stack, no
// counters), with 2K - 1 contribution slots per lane.
static bool retro_of(const PingArgs &a) { return (a.flags & FLAG_RETRO_CHAIN) && a.K > 1; }

hipError_t launch_ping(const PingArgs &a, int stack_depth, hipStream_t s)
{
    int64_t threads = (int64_t)a.n_beams * a.n_r;
    int nblocks = (int)((threads + BLOCK - 1) / BLOCK);
    if (nblocks == 0) return hipSuccess;
    if (retro_of(a)) {
        const int ww = ping_wave_words(64, a.n_bins, a.K, true);
        const size_t shmem = (size_t)ww * 4 * WAVES_PER_BLOCK;
#define SONAR_LAUNCH_R(KK, AR) \
    hipLaunchKernelGGL((k_ping<64, KK, AR, false, false, true>), dim3(nblocks), dim3(BLOCK), shmem, s, a, ww)
        const bool arc = a.g != 0.0;
        switch (a.K) {
            case 2: if (arc) SONAR_LAUNCH_R(2, true); else SONAR_LAUNCH_R(2, false); break;
            case 3: if (arc) SONAR_LAUNCH_R(3, true); else SONAR_LAUNCH_R(3, false); break;
            default: if (arc) SONAR_LAUNCH_R(4, true); else SONAR_LAUNCH_R(4, false); break;
        }
#undef SONAR_LAUNCH_R
        return hipGetLastError();
    }
    // the counting variants exist for the deep stack only (same results)
    int depth = stack_depth <= 32 && !a.stats ? 32 : 64;
    int ww = ping_wave_words(depth, a.n_bins, a.K);
    size_t shmem = (size_t)ww * 4 * WAVES_PER_BLOCK;
#define SONAR_LAUNCH(D, KK, AR, ST) \
    hipLaunchKernelGGL((k_ping<D, KK, AR, ST>), dim3(nblocks), dim3(BLOCK), shmem, s, a, ww)
#define SONAR_LAUNCH_K(D, AR, ST)                     \
    switch (a.K) {                                    \
        case 1: SONAR_LAUNCH(D, 1, AR, ST); break;    \
        case 2: SONAR_LAUNCH(D, 2, AR, ST); break;    \
        case 3: SONAR_LAUNCH(D, 3, AR, ST); break;    \
        default: SONAR_LAUNCH(D, 4, AR, ST); break;   \
    }
    const bool arc = a.g != 0.0;
    if (a.stats) {
        if (arc) { SONAR_LAUNCH_K(64, true, true) } else { SONAR_LAUNCH_K(64, false, true) }
    } else if (depth == 32) {
        if (arc) { SONAR_LAUNCH_K(32, true, false) } else { SONAR_LAUNCH_K(32, false, false) }
    } else {
        if (arc) { SONAR_LAUNCH_K(64, true, false) } else { SONAR_LAUNCH_K(64, false, false) }
    }
#undef SONAR_LAUNCH_K
#undef SONAR_LAUNCH
    return hipGetLastError();
}

hipError_t launch_ping_layered(const PingArgs &a, int stack_depth, hipStream_t s)
{
    int64_t threads = (int64_t)a.n_beams * a.n_r;
    int nblocks = (int)((threads + BLOCK - 1) / BLOCK);
    if (nblocks == 0) return hipSuccess;
    if (retro_of(a)) {
        const int ww = ping_wave_words(64, a.n_bins, a.K, true);
        const size_t shmem = (size_t)ww * 4 * WAVES_PER_BLOCK;
        switch (a.K) {
            case 2: hipLaunchKernelGGL((k_ping<64, 2, true, false, true, true>), dim3(nblocks), dim3(BLOCK), shmem, s, a, ww); break;
            case 3: hipLaunchKernelGGL((k_ping<64, 3, true, false, true, true>), dim3(nblocks), dim3(BLOCK), shmem, s, a, ww); break;
            default: hipLaunchKernelGGL((k_ping<64, 4, true, false, true, true>), dim3(nblocks), dim3(BLOCK), shmem, s, a, ww); break;
        }
        return hipGetLastError();
    }
    int depth = stack_depth <= 32 && !a.stats ? 32 : 64;
    int ww = ping_wave_words(depth, a.n_bins, a.K);
    size_t shmem = (size_t)ww * 4 * WAVES_PER_BLOCK;
#define SONAR_LAUNCH(D, KK, ST) \
    hipLaunchKernelGGL((k_ping<D, KK, true, ST, true>), dim3(nblocks), dim3(BLOCK), shmem, s, a, ww)
#define SONAR_LAUNCH_K(D, ST)                     \
    switch (a.K) {                                \
        case 1: SONAR_LAUNCH(D, 1, ST); break;    \
        case 2: SONAR_LAUNCH(D, 2, ST); break;    \
        case 3: SONAR_LAUNCH(D, 3, ST); break;    \
        default: SONAR_LAUNCH(D, 4, ST); break;   \
    }
    if (a.stats) {
        SONAR_LAUNCH_K(64, true)
    } else if (depth == 32) {
        SONAR_LAUNCH_K(32, false)
    } else {
        SONAR_LAUNCH_K(64, false)
    }
#undef SONAR_LAUNCH_K
#undef SONAR_LAUNCH
    return hipGetLastError();
}

template <int D, int KK, bool AR, bool LAY = false, bool RET = false, int WPB = WAVES_PER_BLOCK>
static hipError_t batch_go(const BatchLaunch &b, hipStream_t s, bool query, int *occ)
{
    const int ww = ping_wave_words(D, b.max_bins, KK, RET);
    const int threads = WPB * WAVE;
    const size_t shmem = (size_t)ww * 4 * WPB;
    const void *kern = reinterpret_cast<const void *>(k_ping_batch<D, KK, AR, LAY, RET, WPB>);
    if (query) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, threads, shmem);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int per_cu = b.blocks_per_cu;
    if (per_cu <= 0) {
        int o = 1;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kern, threads, shmem);
        if (e != hipSuccess) return e;
        per_cu = o > 0 ? o : 1;
    }
    const int tpi = b.tiles_per_item > 0 ? b.tiles_per_item : 1;
    const int64_t units = b.total_tiles * (WAVES_PER_BLOCK / WPB);
    const int64_t items = (units + tpi - 1) / tpi;
    int64_t grid = (int64_t)cus * per_cu;
    if (grid > items) grid = items;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_batch_reset, dim3((b.n_pings + 255) / 256), dim3(256), 0, s, b.queue, b.t0, b.t1,
                       b.n_pings);
    if (b.rx) hipLaunchKernelGGL(k_rx_reset_batch, dim3((b.n_pings + 255) / 256), dim3(256), 0, s, b.desc, b.n_pings);
    hipLaunchKernelGGL((k_ping_batch<D, KK, AR, LAY, RET, WPB>), dim3((unsigned)grid), dim3(threads), shmem, s, b.desc,
                       b.n_pings, b.queue, b.t0, b.t1, ww, tpi);
    if (b.rx)
        hipLaunchKernelGGL(k_rx_scatter_batch, dim3(64, (unsigned)(b.n_pings < 4096 ? b.n_pings : 4096)), dim3(256), 0,
                           s, b.desc, b.n_pings);
    return hipGetLastError();
}

// The workgroup size knob (1, 2 or 4 waves) of the common instantiations.
template <int D, int KK, bool AR>
static hipError_t batch_go_wpb(const BatchLaunch &b, hipStream_t s, bool query, int *occ)
{
    switch (b.waves_per_block) {
        case 1: return batch_go<D, KK, AR, false, false, 1>(b, s, query, occ);
        case 2: return batch_go<D, KK, AR, false, false, 2>(b, s, query, occ);
        default: return batch_go<D, KK, AR, false, false, 4>(b, s, query, occ);
    }
}

static hipError_t batch_dispatch(const BatchLaunch &b, hipStream_t s, bool query, int *occ)
{
#define SONAR_BK(D, AR)                                           \
    switch (b.K) {                                                \
        case 1: return batch_go_wpb<D, 1, AR>(b, s, query, occ);  \
        case 2: return batch_go_wpb<D, 2, AR>(b, s, query, occ);  \
        case 3: return batch_go_wpb<D, 3, AR>(b, s, query, occ);  \
        default: return batch_go_wpb<D, 4, AR>(b, s, query, occ); \
    }
    if (b.retro && b.K > 1) {
        // retro-chain returns: their own instantiations (deep stack, 2K - 1 slots)
        if (b.layered) {
            switch (b.K) {
                case 2: return batch_go<64, 2, true, true, true>(b, s, query, occ);
                case 3: return batch_go<64, 3, true, true, true>(b, s, query, occ);
                default: return batch_go<64, 4, true, true, true>(b, s, query, occ);
            }
        }
        switch (b.K) {
            case 2: return b.arc ? batch_go<64, 2, true, false, true>(b, s, query, occ)
                                 : batch_go<64, 2, false, false, true>(b, s, query, occ);
            case 3: return b.arc ? batch_go<64, 3, true, false, true>(b, s, query, occ)
                                 : batch_go<64, 3, false, false, true>(b, s, query, occ);
            default: return b.arc ? batch_go<64, 4, true, false, true>(b, s, query, occ)
                                  : batch_go<64, 4, false, false, true>(b, s, query, occ);
        }
    }
    if (b.layered) {
        // a batch through one layered profile: the deep-stack instantiations
        switch (b.K) {
            case 1: return batch_go<64, 1, true, true>(b, s, query, occ);
            case 2: return batch_go<64, 2, true, true>(b, s, query, occ);
            case 3: return batch_go<64, 3, true, true>(b, s, query, occ);
            default: return batch_go<64, 4, true, true>(b, s, query, occ);
        }
    }
    if (b.depth <= 32) {
        if (b.arc) { SONAR_BK(32, true) } else { SONAR_BK(32, false) }
    } else {
        if (b.arc) { SONAR_BK(64, true) } else { SONAR_BK(64, false) }
    }
#undef SONAR_BK
}

hipError_t launch_ping_batch(const BatchLaunch &b, hipStream_t s)
{
    if (b.n_pings <= 0 || b.total_tiles <= 0) return hipSuccess;
    return batch_dispatch(b, s, false, nullptr);
}

int batch_max_blocks_per_cu(const BatchLaunch &b)
{
    int occ = 1;
    if (batch_dispatch(b, nullptr, true, &occ) != hipSuccess) return 1;
    return occ > 0 ? occ : 1;
}

}  // namespace sonar
