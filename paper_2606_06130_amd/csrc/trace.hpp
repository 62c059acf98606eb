// Core of ray tracing shared by the ping kernels: FP64 vector helpers,
// triangle records, exact circular-arc paths of a linear sound-speed
// gradient (Sec. II-A: Snell's law), conservative FP32 slab tests,
// Moller-Trumbore and arc-triangle tests, stack traversal of the 4-wide
// hierarchy, FP64 re-intersection, the connection (eigenray) to the sensor,
// drawn continuations, receive-binning lists, and the per-wave fixed-order
// reduction of contributions into beam columns with the fused CFAR test
// (Sec. II-B: coherent summation within each ray bundle). Each translation
// unit that includes it gets its own copy (an anonymous namespace).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.hpp"

namespace sonar {

namespace {

constexpr int WAVE = 64;
constexpr int WAVES_PER_BLOCK = 4;
constexpr int BLOCK = WAVE * WAVES_PER_BLOCK;
constexpr double EPS_SELF = 1e-4;        // minimum hit distance (m)
constexpr double TWO_PI = 6.283185307179586476925287;
constexpr double LN10_OVER_20 = 0.11512925464970228420;

// Single-bounce LDS words per wave for the accumulation stage (one slot per
// lane: bin, value; then the uint16 column index). The area is shared with
// the traversal stack, which is dead by then.
constexpr int K1_BIN_WORDS = WAVE;                            // int bin per slot
constexpr int K1_VAL_WORDS = WAVE * 4;                        // float4 per slot
constexpr int K1_IDX_BASE = K1_BIN_WORDS + K1_VAL_WORDS;      // uint16 column index
// Traversals keep the bottom entries of each lane's stack in LDS (20 for a
// single bounce, 32 with several) and deeper ones in private memory. Typical
// traversals stay in LDS; the short LDS stack is what lets eight waves share
// a SIMD.
constexpr int K1_LDS_STACK = 20;
constexpr int KN_LDS_STACK = 32;
// LDS stack entries with retro-chain slots (2K - 1 per lane): three bounces
// keep three blocks per CU (160 KB), four bounces keep a block within 64 KB;
// the column index reuses the stack, so it holds up to entries * 64 * 2 bins
constexpr int kn_lds_stack_retro(int K) { return K == 3 ? 26 : (K == 4 ? 28 : KN_LDS_STACK); }

struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 mk3(double x, double y, double z) { return d3{x, y, z}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ d3 operator*(d3 a, double s) { return mk3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ double dot3(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross3(d3 a, d3 b)
{
    return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double norm3(d3 a) { return sqrt(dot3(a, a)); }

__device__ __forceinline__ float3 f3(d3 a) { return make_float3((float)a.x, (float)a.y, (float)a.z); }
__device__ __forceinline__ float3 fsub(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float fdot(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 fcross(float3 a, float3 b)
{
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Wavefront-scope barrier for LDS regions private to one wave.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Scene arrays as global-memory pointers: a pointer read from a batch
// descriptor is otherwise generic and its loads become flat loads.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
using gchar = __attribute__((address_space(1))) const char;
__device__ __forceinline__ gchar *as_global(const float4 *p) { return (gchar *)p; }
__device__ __forceinline__ float4 ldg4(gchar *p)
{
    const f4v v = *(__attribute__((address_space(1))) const f4v *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

// Triangle record -> vertices, id bits.
struct TriF {
    float3 v0, v1, v2;
    uint32_t idbits;
    float rho, phi;
};
__device__ __forceinline__ TriF load_tri(gchar *__restrict__ tris, uint32_t i)
{
    gchar *r = tris + 48 * (size_t)i;
    const float4 a = ldg4(r), b = ldg4(r + 16), c = ldg4(r + 32);
    TriF t;
    t.v0 = make_float3(a.x, a.y, a.z);
    t.v1 = make_float3(a.w, b.x, b.y);
    t.v2 = make_float3(b.z, b.w, c.x);
    t.idbits = __float_as_uint(c.y);
    t.rho = c.z;
    t.phi = c.w;
    return t;
}

// ---------------------------------------------------------------------------
// Paths. In c(z) = c0 + g z the Snell invariant cos(theta) / c is constant and
// a ray is a circle of curvature kappa = g cos(theta) / c(z) centred on the
// plane c = 0: x(s) = o + d sin(ks)/k + nc (1 - cos ks)/k, with nc the unit
// normal toward the centre in the ray's vertical plane. With g = 0 or a
// vertical direction the path is straight.
struct Path64 {
    d3 o, d, nc;
    double kappa;
    bool arc;
};

__device__ __forceinline__ Path64 make_path(d3 o, d3 d, double g, double c0)
{
    Path64 p;
    p.o = o;
    p.d = d;
    p.arc = false;
    p.kappa = 0.0;
    p.nc = mk3(0.0, 0.0, 0.0);
    double dh = sqrt(d.x * d.x + d.y * d.y);
    if (g != 0.0 && dh > 0.0) {
        p.arc = true;
        p.kappa = g * dh / (c0 + g * o.z);
        p.nc = mk3(d.z * d.x / dh, d.z * d.y / dh, -dh);
    }
    return p;
}

__device__ __forceinline__ d3 path_point(const Path64 &p, double s)
{
    if (!p.arc) return p.o + p.d * s;
    double u = p.kappa * s, h = sin(0.5 * u);
    return p.o + p.d * (sin(u) / p.kappa) + p.nc * (2.0 * h * h / p.kappa);
}

__device__ __forceinline__ d3 path_tangent(const Path64 &p, double s)
{
    if (!p.arc) return p.d;
    double u = p.kappa * s;
    return p.d * cos(u) + p.nc * sin(u);
}

// One-way time along the path. On the arc, dt = ds / c and the integral from
// grazing angle th0 to th1 is (atanh sin th0 - atanh sin th1) / g, evaluated
// here as one atanh of (s0 - s1) / (1 - s0 s1) with s0 - s1 and
// 1 - s0 s1 = cos^2 th0 + s0 (s0 - s1) formed without cancellation.
__device__ __forceinline__ double path_time(const Path64 &p, double s, double g, double c0)
{
    if (!p.arc) {
        if (g == 0.0) return s / c0;
        return fabs(log1p(g * p.d.z * s / (c0 + g * p.o.z)) / g);   // vertical ray
    }
    double u = p.kappa * s, h = sin(0.5 * u);
    double dh = sqrt(p.d.x * p.d.x + p.d.y * p.d.y);
    double s0 = p.d.z;
    double ds = p.d.z * 2.0 * h * h + dh * sin(u);                   // sin th0 - sin th1
    return atanh(ds / (dh * dh + s0 * ds)) / g;
}

// FP32 traversal segment: a straight ray, or for an arc the chord from o to
// x(s_lim) with node boxes inflated by the arc's largest distance to it.
struct Seg32 {
    float3 o, d, inv;      // the ray or the chord
    float sigma;           // box inflation (0 for straight rays)
    float tmin, tmax;      // parameter range on the ray or chord
    float smin, smax;      // arc-length range of valid hits
    float3 ad, anc;        // arc tangent and centre normal at o
    float kappa;
};

__device__ __forceinline__ float3 safe_inv(float3 d)
{
    // zero components get a tiny signed value so that slab distances stay finite or infinite, never NaN
    float dx = fabsf(d.x) > 1e-30f ? d.x : copysignf(1e-30f, d.x);
    float dy = fabsf(d.y) > 1e-30f ? d.y : copysignf(1e-30f, d.y);
    float dz = fabsf(d.z) > 1e-30f ? d.z : copysignf(1e-30f, d.z);
    return make_float3(1.0f / dx, 1.0f / dy, 1.0f / dz);
}

__device__ __forceinline__ Seg32 make_seg(const Path64 &p, double smin, double smax)
{
    Seg32 g;
    g.o = f3(p.o);
    g.smin = (float)smin;
    g.smax = (float)smax;
    if (!p.arc) {
        g.d = f3(p.d);
        g.sigma = 0.f;
        g.tmin = (float)smin;
        g.tmax = (float)smax;
        g.kappa = 0.f;
        g.ad = g.d;
        g.anc = make_float3(0.f, 0.f, 0.f);
    } else {
        d3 e = path_point(p, smax) - p.o;
        double lc = norm3(e);
        g.d = f3(e * (1.0 / lc));
        // sagitta of the arc over its chord, with margin for FP32 rounding of the chord
        double sag = fabs(p.kappa) * smax * smax / 8.0;
        g.sigma = (float)(sag * 1.01 + 2e-6 * (1.0 + smax));
        g.tmin = 0.f;
        g.tmax = (float)(lc * (1.0 + 1e-6));
        g.kappa = (float)p.kappa;
        g.ad = f3(p.d);
        g.anc = f3(p.nc);
    }
    g.inv = safe_inv(g.d);
    return g;
}

// Per-traversal constants of the slab test. For each axis the plane a ray
// enters first (near) is the lower one when the inverse direction is >= 0,
// else the upper one; the node stores lower and upper planes of an axis in
// adjacent 16-byte rows, so the near and far rows are picked by a per-lane
// byte offset and no min/max per axis is needed. A plane distance is one FMA,
// t = p * inv + c, with c = -(o * inv) rounded and then widened by 2^-21 |o *
// inv| (eight roundings of the product): every near distance comes out no
// later and every far distance no earlier than with exact arithmetic on
// these operands, which amounts to growing the box by 2^-21 |o| along each
// axis. Curved rays test the box inflated by the sagitta s: lower planes
// against o + s, upper planes against o - s.
struct SlabRay {
    float3 inv, cn, cf;       // inverse direction, near and far constants
    uint32_t ox, oy, oz;      // byte offsets of the near rows (far row: offset ^ 16)
};

__device__ __forceinline__ void slab_axis(float o, float s, float inv, uint32_t base, uint32_t &off, float &cn,
                                          float &cf)
{
    const bool neg = __float_as_uint(inv) >> 31;
    off = base | (neg ? 16u : 0u);
    const float on = neg ? o - s : o + s, of = neg ? o + s : o - s;
    const float an = on * inv, af = of * inv;
    cn = -an - fabsf(an) * 0x1p-21f;
    cf = -af + fabsf(af) * 0x1p-21f;
}

__device__ __forceinline__ SlabRay slab_ray(const float3 &o, const float3 &inv, float sigma)
{
    SlabRay q;
    q.inv = inv;
    slab_axis(o.x, sigma, inv.x, 0u, q.ox, q.cn.x, q.cf.x);
    slab_axis(o.y, sigma, inv.y, 32u, q.oy, q.cn.y, q.cf.y);
    slab_axis(o.z, sigma, inv.z, 64u, q.oz, q.cn.z, q.cf.z);
    return q;
}

// One child box against [tmin, tmax] from its near and far planes; the far
// distance is widened by 5e-7 relative for the rounding of the FMA results
// and of the inverse direction.
__device__ __forceinline__ bool slab(const SlabRay &q, float nx, float ny, float nz, float fx, float fy, float fz,
                                     float tmin, float tmax, float &tnear)
{
    const float tn = fmaxf(fmaxf(fmaf(nx, q.inv.x, q.cn.x), fmaf(ny, q.inv.y, q.cn.y)),
                           fmaxf(fmaf(nz, q.inv.z, q.cn.z), tmin));
    const float tf = fminf(fminf(fmaf(fx, q.inv.x, q.cf.x), fmaf(fy, q.inv.y, q.cf.y)),
                           fminf(fmaf(fz, q.inv.z, q.cf.z), tmax));
    tnear = tn;
    return tn <= tf * 1.0000005f;
}

// FP32 Moller-Trumbore (closed triangle), without a division on the
// barycentric tests: with U = u det and V = v det the hit is inside when U, V
// and det - U - V share det's sign. Returns t or -1.
__device__ __forceinline__ float mt32(const Seg32 &r, const TriF &t)
{
    const float3 e1 = fsub(t.v1, t.v0), e2 = fsub(t.v2, t.v0);
    const float3 p = fcross(r.d, e2);
    const float det = fdot(e1, p);
    const float3 tv = fsub(r.o, t.v0);
    const float U = fdot(tv, p);
    const float3 q = fcross(tv, e1);
    const float V = fdot(r.d, q);
    const float W = U + V;
    const bool in = det > 0.f ? (U >= 0.f && V >= 0.f && W <= det) : (det < 0.f && U <= 0.f && V <= 0.f && W >= det);
    if (!in) return -1.f;
    return fdot(e2, q) / det;
}

// FP32 arc-triangle test: smallest arc length s in (smin, smax] where the arc
// meets the triangle's plane inside the closed triangle; -1 if none. The
// plane equation f(s) = n.(o - v0) + n.d S(s) + n.nc C(s), with S = sin(ks)/k
// and C = (1 - cos ks)/k, is solved to second order in k s (stable quadratic
// formula) and then polished by one Newton step with the third-order terms.
// `tc` returns the hit's parameter along the chord, used for culling.
__device__ __forceinline__ float arc32(const Seg32 &r, const TriF &t, float &tc)
{
    float3 e1 = fsub(t.v1, t.v0), e2 = fsub(t.v2, t.v0);
    float3 n = fcross(e1, e2);
    float3 ov = fsub(r.o, t.v0);
    const float k = r.kappa;
    float fa = fdot(n, ov), fb = fdot(n, r.ad), fn = fdot(n, r.anc);
    float fc = 0.5f * fn * k;
    float s0 = -1.f, s1 = -1.f;
    if (fc == 0.f) {
        if (fb != 0.f) s0 = -fa / fb;
    } else {
        float disc = fb * fb - 4.f * fc * fa;
        if (disc < 0.f) return -1.f;
        float sq = sqrtf(disc);
        float q = -0.5f * (fb + (fb >= 0.f ? sq : -sq));
        s0 = q / fc;
        s1 = q != 0.f ? fa / q : -1.f;
        if (s1 < s0) { float w = s0; s0 = s1; s1 = w; }
    }
    float nn = fdot(n, n);
    for (int m = 0; m < 2; ++m) {
        float s = m == 0 ? s0 : s1;
        if (!(s > 0.f)) continue;
        {   // Newton step with the cubic terms of S and C
            float ks = k * s;
            float Ss = s * (1.f - ks * ks * (1.f / 6.f));
            float Cs = 0.5f * ks * s * (1.f - ks * ks * (1.f / 12.f));
            float f = fa + fb * Ss + fn * Cs;
            float fp = fb * (1.f - 0.5f * ks * ks) + fn * ks * (1.f - ks * ks * (1.f / 6.f));
            if (fp != 0.f) s -= f / fp;
        }
        if (!(s > r.smin && s <= r.smax)) continue;
        float ks = k * s;
        float Ss = s * (1.f - ks * ks * (1.f / 6.f));
        float Cs = 0.5f * ks * s * (1.f - ks * ks * (1.f / 12.f));
        float3 x = make_float3(ov.x + r.ad.x * Ss + r.anc.x * Cs, ov.y + r.ad.y * Ss + r.anc.y * Cs,
                               ov.z + r.ad.z * Ss + r.anc.z * Cs);
        float u = fdot(fcross(x, e2), n), v = fdot(fcross(e1, x), n);
        if (u >= 0.f && v >= 0.f && u + v <= nn) {
            float3 xw = make_float3(x.x + t.v0.x - r.o.x, x.y + t.v0.y - r.o.y, x.z + t.v0.z - r.o.z);
            tc = fdot(xw, r.d);
            return s;
        }
    }
    return -1.f;
}

// Stack-based BVH traversal (near child first). ANY = true returns at the
// first valid hit. `skip` is an original triangle index never reported.
// Returns the triangle record index, or -1; `overflow` is set when the LDS
// stack of DEPTH entries would overflow or the node-visit bound is reached
// (the ray is then reported as a miss).
// Orders two (distance, link) pairs by distance (ties keep their order).
__device__ __forceinline__ void order2(float &ta, uint32_t &la, float &tb, uint32_t &lb)
{
    const bool sw = tb < ta;
    const float t = sw ? tb : ta;
    tb = sw ? ta : tb;
    ta = t;
    const uint32_t l = sw ? lb : la;
    lb = sw ? la : lb;
    la = l;
}

// Nearest-hit (or any-hit) traversal of the 4-wide hierarchy. An inner node
// tests its four child boxes, descends into the nearest one hit and pushes
// the others farthest first; leaves test their triangles. The stack keeps
// its bottom DL entries of each lane in LDS, deeper ones in private memory.
template <int DEPTH, int DL, bool ANY, bool ARC, bool STATS>
__device__ int traverse(gchar *__restrict__ nodes, gchar *__restrict__ tris, const Seg32 &r,
                        uint32_t skip, uint32_t *__restrict__ stk, int lane, bool &overflow, float &s_out,
                        uint32_t max_steps, uint32_t &n_nodes, uint32_t &n_tris, uint32_t &n_deep)
{
    constexpr float MISS = __builtin_inff();
    int best = -1;
    float best_t = r.tmax;        // culling bound on the ray / chord parameter
    float best_s = r.smax;        // best arc length
    uint32_t best_id = 0xFFFFFFFFu;
    const float sg = r.sigma;
    const SlabRay q = slab_ray(r.o, r.inv, sg);
    uint32_t cur = 0;
    int sp = 0;
    // entries sp >= DL: private memory (volatile keeps them out of registers)
    volatile uint32_t spill[DEPTH > DL ? DEPTH - DL : 1];
    for (uint32_t step = 0;; ++step) {
        if (step >= max_steps) {   // bound on node visits: every wave exits
            overflow = true;
            best = -1;
            break;
        }
        if (!(cur & LEAF_BIT)) {
            if (STATS) ++n_nodes;
            // 32-bit byte offsets into the node array (at most 2^25 nodes)
            const uint32_t at = cur << 7, nx_at = at | q.ox, ny_at = at | q.oy, nz_at = at | q.oz;
            const float4 nx = ldg4(nodes + nx_at);
            const float4 fx = ldg4(nodes + (nx_at ^ 16u));
            const float4 ny = ldg4(nodes + ny_at);
            const float4 fy = ldg4(nodes + (ny_at ^ 16u));
            const float4 nz = ldg4(nodes + nz_at);
            const float4 fz = ldg4(nodes + (nz_at ^ 16u));
            const float4 lk = ldg4(nodes + (at | 96u));
            float t0, t1, t2, t3;
            const bool h0 = slab(q, nx.x, ny.x, nz.x, fx.x, fy.x, fz.x, r.tmin, best_t, t0);
            const bool h1 = slab(q, nx.y, ny.y, nz.y, fx.y, fy.y, fz.y, r.tmin, best_t, t1);
            const bool h2 = slab(q, nx.z, ny.z, nz.z, fx.z, fy.z, fz.z, r.tmin, best_t, t2);
            const bool h3 = slab(q, nx.w, ny.w, nz.w, fx.w, fy.w, fz.w, r.tmin, best_t, t3);
            float ta = h0 ? t0 : MISS, tb = h1 ? t1 : MISS, tc = h2 ? t2 : MISS, td = h3 ? t3 : MISS;
            uint32_t la = __float_as_uint(lk.x), lb = __float_as_uint(lk.y), lc = __float_as_uint(lk.z),
                     ld = __float_as_uint(lk.w);
            order2(ta, la, tb, lb);
            order2(tc, lc, td, ld);
            order2(ta, la, tc, lc);
            order2(tb, lb, td, ld);
            order2(tb, lb, tc, lc);
            if (ta != MISS) {
                const int np = (tb != MISS) + (tc != MISS) + (td != MISS);
                if (sp + np > DEPTH) {
                    overflow = true;
                    best = -1;
                    break;
                }
                // the np links to push, farthest first, are the last np of (ld, lc, lb)
                const uint32_t p0 = np == 3 ? ld : (np == 2 ? lc : lb);
                const uint32_t p1 = np == 3 ? lc : lb;
                if (sp + 3 <= DL) {
                    // common case: three LDS slots written unconditionally
                    // (entries past the new top are never read)
                    stk[sp * WAVE + lane] = p0;
                    stk[(sp + 1) * WAVE + lane] = p1;
                    stk[(sp + 2) * WAVE + lane] = lb;
                    sp += np;
                } else {
                    const uint32_t lp[3] = {p0, p1, lb};
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        if (q < np) {
                            if (DL == DEPTH || sp < DL) stk[sp * WAVE + lane] = lp[q];
                            else spill[sp - DL] = lp[q];
                            ++sp;
                        }
                    }
                }
                if (STATS) n_deep = max(n_deep, (uint32_t)sp);
                cur = la;
                continue;
            }
        } else if (cur != EMPTY_LINK) {
            uint32_t first = (cur & 0x7FFFFFFFu) >> 3;
            uint32_t cnt = (cur & 7u) + 1u;
            if (STATS) n_tris += cnt;
            for (uint32_t k = 0; k < cnt; ++k) {
                TriF t = load_tri(tris, first + k);
                uint32_t id = t.idbits & 0x7FFFFFFFu;
                if (id == skip) continue;
                float sh, th;
                if (ARC) {
                    sh = arc32(r, t, th);
                    if (sh < 0.f) continue;
                } else {
                    sh = mt32(r, t);
                    th = sh;
                    if (!(sh > r.smin)) continue;
                }
                if (sh < best_s || (sh == best_s && id < best_id)) {
                    best = (int)(first + k);
                    best_s = sh;
                    best_t = ARC ? fminf(best_t, th + 2.f * sg) : sh;
                    best_id = id;
                    if (ANY) break;
                }
            }
            if (ANY && best >= 0) break;
        }
        if (sp == 0) break;
        --sp;
        if (DL == DEPTH || sp < DL) cur = stk[sp * WAVE + lane];
        else cur = spill[sp - DL];
    }
    s_out = best_s;
    return best;
}

// FP64 re-intersection of a triangle record along a path: Moller-Trumbore for
// a straight path, Newton on the plane equation of the exact arc otherwise.
__device__ __forceinline__ double refine64(const TriF &t, const Path64 &p, double s_guess, d3 &nrm)
{
    d3 v0 = mk3(t.v0.x, t.v0.y, t.v0.z), v1 = mk3(t.v1.x, t.v1.y, t.v1.z), v2 = mk3(t.v2.x, t.v2.y, t.v2.z);
    d3 e1 = v1 - v0, e2 = v2 - v0;
    d3 n = cross3(e1, e2);
    nrm = n * (1.0 / norm3(n));
    if (!p.arc) {
        d3 q = cross3(p.o - v0, e1);
        d3 pv = cross3(p.d, e2);
        return dot3(e2, q) / dot3(e1, pv);
    }
    double s = s_guess;
    for (int it = 0; it < 4; ++it) {
        double f = dot3(nrm, path_point(p, s) - v0);
        double fp = dot3(nrm, path_tangent(p, s));
        if (fp == 0.0) break;
        s -= f / fp;
    }
    return s;
}

__device__ __forceinline__ int xcd_remap(int bid, int nblocks)
{
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of tiles so that neighbouring beams share one L2.
    const int X = 8;
    int x = bid % X, i = bid / X;
    int q = nblocks / X, rmd = nblocks % X;
    return x * q + min(x, rmd) + i;
}

struct Slot {
    int bin;
    float re, im, inc;
};

// Connection from a scattering point P back to the sensor at S: a straight
// segment when g = 0, else the circle through both points with its centre on
// the plane c = 0 in their vertical plane (the eigenray).
struct Conn {
    double L, T;
    d3 w;          // departure direction at P
    d3 arrive;     // direction of travel at S
};

__device__ __forceinline__ Conn connect(d3 P, d3 S, double g, double c0)
{
    Conn c;
    d3 v = S - P;
    double D = sqrt(v.x * v.x + v.y * v.y);
    if (g == 0.0 || D == 0.0) {
        c.L = norm3(v);
        c.w = v * (1.0 / c.L);
        c.arrive = c.w;
        c.T = g == 0.0 ? c.L / c0 : fabs(log1p(g * v.z / (c0 + g * P.z)) / g);
        return c;
    }
    // heights above the centre plane in a frame where the gradient is positive
    const double sg = g > 0.0 ? 1.0 : -1.0, ag = fabs(g);
    const double zc = -c0 / ag;
    const double h1 = sg * P.z - zc, h2 = sg * S.z - zc;
    // centre at horizontal distance xc from P toward S on the perpendicular bisector
    const double xc = 0.5 * D + 0.5 * (h2 - h1) * (h2 + h1) / D;
    const double R = sqrt(xc * xc + h1 * h1);
    const d3 uh = mk3(v.x / D, v.y / D, 0.0);
    const double sin0 = xc / R, cos0 = h1 / R, sin1 = (xc - D) / R, cos1 = h2 / R;
    c.w = mk3(cos0 * uh.x, cos0 * uh.y, sg * sin0);
    c.arrive = mk3(cos1 * uh.x, cos1 * uh.y, sg * sin1);
    c.L = 2.0 * R * asin(0.5 * norm3(v) / R);
    const double dsn = D / R;                        // sin0 - sin1
    c.T = atanh(dsn / (cos0 * cos0 + sin0 * dsn)) / ag;
    return c;
}


// Monte-Carlo continuation after a rough facet: the Phong lobe around the
// mirror direction with probability k_s / (k_d + k_s), else the cosine lobe
// around the facet normal facing the ray; uniforms from SplitMix64 output
// c + 1 of (seed xor 0xD1B54A32D192ED03), c = (ping << 40) ^ (ray << 2) ^ k,
// azimuth in the orthonormal basis of Duff et al. (JCGT 2017). `lit` is false
// when the drawn direction does not leave the lit side. Kept out of line
// (scalar arguments, result by value) so that the kernels that never draw
// keep their register allocation.
struct Drawn {
    d3 dir;
    bool lit;
};

__device__ __attribute__((noinline)) Drawn draw_continuation(const uint64_t seed, const uint32_t ping,
                                                             const double phong_n, const uint64_t ray, const int k,
                                                             const d3 rh, const d3 np, const double kd,
                                                             const double ks)
{
    const uint64_t c = ((uint64_t)ping << 40) ^ (ray << 2) ^ (uint64_t)k;
    const uint64_t z = splitmix64_nth(seed ^ 0xD1B54A32D192ED03ull, c + 1);
    const double u1 = (double)(z >> 40) * (1.0 / 16777216.0);
    const double u2 = (double)((z >> 16) & 0xFFFFFFull) * (1.0 / 16777216.0);
    const double u3 = (double)(z & 0xFFFFull) * (1.0 / 65536.0);
    const bool spec = u3 < ks / (kd + ks);
    const d3 ax = spec ? rh : np;
    const double ca = spec ? pow(1.0 - u1, 1.0 / (phong_n + 1.0)) : sqrt(1.0 - u1);
    const double sa = sqrt(fmax(0.0, 1.0 - ca * ca)), ph = TWO_PI * u2;
    const double sg = ax.z >= 0.0 ? 1.0 : -1.0, q = -1.0 / (sg + ax.z), b = ax.x * ax.y * q;
    const d3 t1 = mk3(1.0 + sg * ax.x * ax.x * q, sg * b, -sg * ax.x), t2 = mk3(b, sg + ax.y * ax.y * q, -ax.y);
    const d3 v = ax * ca + t1 * (sa * cos(ph)) + t2 * (sa * sin(ph));
    Drawn r;
    r.dir = v * (1.0 / norm3(v));
    r.lit = dot3(r.dir, np) > 0.0;
    return r;
}

// Receive binning: a return added to another beam than the launch beam is
// appended to a device list, one counter update per wave (ballot, the
// leader's atomic, per-lane offsets from the lanes below).
__device__ __forceinline__ void rx_append(const PingArgs &a, const bool want, const int4 e, const int lane)
{
    const uint64_t m = __ballot(want);
    if (m == 0) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(a.rx_count, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, leader);
    if (want) {
        const uint32_t slot = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (slot < a.rx_cap) a.rx_list[slot] = e;
        else atomicOr(a.status, ST_RX_FULL);
    }
}

// Fixed-order reduction of one wave's contribution slots and the column
// write (with the fused CFAR test when it is on). Slot (k, lane) holds bin
// sbin[k * 64 + lane] and value sval[k * 64 + lane] = (re, im, first-bounce
// |A|^2, later-bounce |A|^2); lanes hold the rays of 64 / n_r beams in order.
// `sidx32` is an LDS area of (n_bins + 1) / 2 words for the column index;
// `ray0` is the block's first ray. Every lane of the wave calls it.
template <int KS>
__device__ __forceinline__ void reduce_tile(const PingArgs &a, const int64_t ray0, const int wave, const int lane,
                                            const int j, const bool active, int *sbin,
                                            float4 *sval, uint32_t *sidx32)
{
    uint16_t *sidx = reinterpret_cast<uint16_t *>(sidx32);
    int my_bin[2 * MAX_BOUNCES - 1];
#pragma unroll
    for (int k = 0; k < KS; ++k) my_bin[k] = sbin[k * WAVE + lane];
    const int nr = a.n_r;
    const int bl = lane >> a.log2_nr;          // beam within the wave
    const int base_lane = bl << a.log2_nr;
    bool head[2 * MAX_BOUNCES - 1];
    float4 sum[2 * MAX_BOUNCES - 1];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        head[k] = false;
        sum[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        int mb = my_bin[k];
        if (mb < 0) continue;
        int me = j * KS + k;
        bool hd = true;
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int jj = 0; jj < nr; ++jj) {
            for (int kk = 0; kk < KS; ++kk) {
                int s2 = kk * WAVE + base_lane + jj;
                if (sbin[s2] != mb) continue;
                int o2 = jj * KS + kk;
                if (o2 < me) {
                    hd = false;
                } else {
                    float4 v = sval[s2];
                    acc.x += v.x;
                    acc.y += v.y;
                    acc.z += v.z;
                    acc.w += v.w;
                }
            }
        }
        head[k] = hd;
        sum[k] = acc;
    }
    wave_sync();
    // from here on a slot that still holds a bin is a head carrying its bin's sum
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        if (head[k]) sval[k * WAVE + lane] = sum[k];
        else sbin[k * WAVE + lane] = -1;
    }
    wave_sync();

    const int bpw = WAVE >> a.log2_nr;
    const int64_t wave_beam0 = (ray0 + wave * WAVE) >> a.log2_nr;
    const int nb = a.n_bins;

    if (a.det_count) {
        // CA-CFAR on the beam's head slots, all beams of the wave at once. A
        // bin without a return has power N0 <= the training mean and alpha(N)
        // > 1, so only bins holding a return can be detected; a training sum
        // is N * N0 plus the excess of the returns inside the window.
        const float n0 = a.det_n0;
        uint64_t key[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            key[k] = 0ull;
            if (!head[k]) continue;
            const int bin = my_bin[k];
            const float4 v = sum[k];
            const float p = v.x * v.x + v.y * v.y + n0;
            const int l0 = max(bin - a.det_G - a.det_T, 0), l1 = max(bin - a.det_G, 0);
            const int h0 = min(bin + a.det_G + 1, nb), h1 = min(bin + a.det_G + a.det_T + 1, nb);
            const int N = (l1 - l0) + (h1 - h0);
            float pl = n0, pr = n0;
            double wsum = (double)N * (double)n0;
            for (int jj = 0; jj < nr; ++jj) {
                for (int kk = 0; kk < KS; ++kk) {
                    const int s2 = kk * WAVE + base_lane + jj;
                    const int b2 = sbin[s2];
                    if (b2 < 0) continue;
                    const bool inw = (b2 >= l0 && b2 < l1) || (b2 >= h0 && b2 < h1);
                    if (!inw && b2 != bin - 1 && b2 != bin + 1) continue;
                    const float4 u = sval[s2];
                    const float pz = u.x * u.x + u.y * u.y + n0;
                    if (b2 == bin - 1) pl = pz;
                    if (b2 == bin + 1) pr = pz;
                    if (inw) wsum += (double)pz - (double)n0;
                }
            }
            if ((bin > 0 && !(p > pl)) || (bin + 1 < nb && !(p >= pr))) continue;
            if (N <= 0) continue;
            const double thr = a.det_alpha[N] * wsum / N;
            if ((double)p > thr) key[k] = ((uint64_t)__float_as_uint(p) << 32) | (uint32_t)(~bin);
        }
        // the det_M strongest of each beam over its lanes, strongest first
        // (every lane of a beam group leaves the loop at the same m)
        const int64_t gb = wave_beam0 + bl;
        unsigned taken = 0u;
        int cnt = 0;
        for (int m = 0; m < a.det_M; ++m) {
            uint64_t my = 0ull;
            int myk = -1;
#pragma unroll
            for (int k = 0; k < KS; ++k)
                if (!((taken >> k) & 1u) && key[k] > my) { my = key[k]; myk = k; }
            uint64_t best = my;
            for (int off = 1; off < nr; off <<= 1) {
                uint64_t o = __shfl_xor(best, off);
                best = o > best ? o : best;
            }
            if (best == 0ull) break;
            if (myk >= 0 && my == best) taken |= 1u << myk;
            if (j == 0 && active) {
                a.det_bins[(size_t)gb * a.det_M + m] = (int)(~(uint32_t)(best & 0xFFFFFFFFu));
                a.det_pw[(size_t)gb * a.det_M + m] = __uint_as_float((uint32_t)(best >> 32));
            }
            cnt = m + 1;
        }
        if (j == 0 && active) a.det_count[gb] = cnt;
    }

    // ---- column write: one beam at a time through the LDS column index, with
    // non-temporal stores (the volume streams out; caching it would evict the
    // hierarchy that the other waves are still traversing)
    const int idx_words = (nb + 1) / 2;
    for (int q = 0; q < bpw; ++q) {
        const int64_t gb = wave_beam0 + q;
        if (gb >= a.n_beams) break;
        for (int w = lane; w < idx_words; w += WAVE) sidx32[w] = 0u;
        wave_sync();
        if (bl == q) {
#pragma unroll
            for (int k = 0; k < KS; ++k)
                if (head[k]) sidx[my_bin[k]] = (uint16_t)(k * WAVE + lane + 1);
        }
        wave_sync();
        float2 *col = a.volume + (size_t)gb * nb;
        float *i1 = a.incoh ? a.incoh + (size_t)gb * nb : nullptr;
        float *im = a.incoh ? a.incoh + ((size_t)a.n_beams + gb) * nb : nullptr;
        if ((nb & 1) == 0) {
            for (int w = lane; w < idx_words; w += WAVE) {
                uint32_t pair = sidx32[w];
                uint32_t s0 = pair & 0xFFFFu, s1 = pair >> 16;
                float4 v0 = s0 ? sval[s0 - 1] : make_float4(0.f, 0.f, 0.f, 0.f);
                float4 v1 = s1 ? sval[s1 - 1] : make_float4(0.f, 0.f, 0.f, 0.f);
                __builtin_nontemporal_store(f4v{v0.x, v0.y, v1.x, v1.y}, reinterpret_cast<f4v *>(col) + w);
                if (i1) {
                    __builtin_nontemporal_store(f2v{v0.z, v1.z}, reinterpret_cast<f2v *>(i1) + w);
                    __builtin_nontemporal_store(f2v{v0.w, v1.w}, reinterpret_cast<f2v *>(im) + w);
                }
            }
        } else {
            for (int b = lane; b < nb; b += WAVE) {
                uint32_t s0 = sidx[b];
                float4 v0 = s0 ? sval[s0 - 1] : make_float4(0.f, 0.f, 0.f, 0.f);
                __builtin_nontemporal_store(f2v{v0.x, v0.y}, reinterpret_cast<f2v *>(col) + b);
                if (i1) {
                    __builtin_nontemporal_store(v0.z, i1 + b);
                    __builtin_nontemporal_store(v0.w, im + b);
                }
            }
        }
        wave_sync();
    }
}

}  // namespace

}  // namespace sonar
