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
// included (coherent summation within each ray bundle, Sec. II-B). No global
// atomics, no memset, bit-reproducible.
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

}  // namespace

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

// The ping body for one tile of 256 consecutive rays (4 wavefronts). `a` is
// the ping's argument block (kernel arguments, or a batch descriptor in
// device memory); `W` is this wavefront's LDS area.
template <int DEPTH, int K, bool ARC, bool STATS, bool LAYERED = false, bool RETRO = false>
__device__ __forceinline__ void ping_tile(const PingArgs &a, const int tile, uint32_t *__restrict__ W)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    const int64_t gid = (int64_t)tile * BLOCK + threadIdx.x;
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
    uint16_t *sidx = reinterpret_cast<uint16_t *>(sidx32);
    if (K == 1) {
        sbin[lane] = slot0.bin;
        sval[lane] = make_float4(slot0.re, slot0.im, slot0.inc, 0.f);
    }
    wave_sync();
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
    const int64_t wave_beam0 = (((int64_t)tile * BLOCK) + wave * WAVE) >> a.log2_nr;
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
        ping_tile<DEPTH, K, ARC, STATS, LAYERED, RETRO>(*ka, xcd_remap(blockIdx.x, gridDim.x), W);
    } else {
        ping_tile<DEPTH, K, ARC, STATS, LAYERED, RETRO>(a, xcd_remap(blockIdx.x, gridDim.x), W);
    }
}

// Persistent batch: every block pops (ping, tile) items from one device
// counter until the queue is empty; per-ping first-start and last-finish
// stamps come from the constant-rate device clock. All pings of a batch share
// the hierarchy depth class, bounce count and medium type (template
// arguments); layouts, rays per beam, poses and outputs come per ping from
// its descriptor.
template <int DEPTH, int K, bool ARC, bool LAYERED = false, bool RETRO = false>
__global__ __attribute__((amdgpu_flat_work_group_size(1, BLOCK), amdgpu_waves_per_eu(ping_waves_per_eu<K, ARC>())))
void k_ping_batch(const PingArgs *__restrict__ desc, int n_pings,
                                                      uint32_t *__restrict__ queue, unsigned long long *__restrict__ t0,
                                                      unsigned long long *__restrict__ t1, int wave_words,
                                                      int tiles_per_item)
{
    extern __shared__ uint32_t lds[];
    __shared__ int s_item;
    uint32_t *W = lds + (size_t)(threadIdx.x / WAVE) * wave_words;
    const PingArgs &last = desc[n_pings - 1];
    const int total_tiles = last.tile_offset + last.n_tiles;
    const int n_items = (total_tiles + tiles_per_item - 1) / tiles_per_item;
    while (true) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);     // uniform: descriptor fields in SGPRs
        __syncthreads();
        if (item >= n_items) break;
        for (int q = 0; q < tiles_per_item; ++q) {
            const int gt = item * tiles_per_item + q;
            if (gt >= total_tiles) break;
            // the ping holding global tile gt: last descriptor with tile_offset <= gt
            int lo = 0, hi = n_pings - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (desc[mid].tile_offset <= gt) lo = mid;
                else hi = mid - 1;
            }
            const PingArgs &a = desc[lo];
            unsigned long long start = __builtin_amdgcn_s_memrealtime();
            ping_tile<DEPTH, K, ARC, false, LAYERED, RETRO>(a, gt - a.tile_offset, W);
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

template <int D, int KK, bool AR, bool LAY = false, bool RET = false>
static hipError_t batch_go(const BatchLaunch &b, hipStream_t s, bool query, int *occ)
{
    const int ww = ping_wave_words(D, b.max_bins, KK, RET);
    const size_t shmem = (size_t)ww * 4 * WAVES_PER_BLOCK;
    if (query) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            occ, reinterpret_cast<const void *>(k_ping_batch<D, KK, AR, LAY, RET>), BLOCK, shmem);
    }
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int per_cu = b.blocks_per_cu;
    if (per_cu <= 0) {
        int o = 1;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &o, reinterpret_cast<const void *>(k_ping_batch<D, KK, AR, LAY, RET>), BLOCK, shmem);
        if (e != hipSuccess) return e;
        per_cu = o > 0 ? o : 1;
    }
    const int tpi = b.tiles_per_item > 0 ? b.tiles_per_item : 1;
    const int64_t items = (b.total_tiles + tpi - 1) / tpi;
    int64_t grid = (int64_t)cus * per_cu;
    if (grid > items) grid = items;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_batch_reset, dim3((b.n_pings + 255) / 256), dim3(256), 0, s, b.queue, b.t0, b.t1,
                       b.n_pings);
    if (b.rx) hipLaunchKernelGGL(k_rx_reset_batch, dim3((b.n_pings + 255) / 256), dim3(256), 0, s, b.desc, b.n_pings);
    hipLaunchKernelGGL((k_ping_batch<D, KK, AR, LAY, RET>), dim3((unsigned)grid), dim3(BLOCK), shmem, s, b.desc, b.n_pings,
                       b.queue, b.t0, b.t1, ww, tpi);
    if (b.rx)
        hipLaunchKernelGGL(k_rx_scatter_batch, dim3(64, (unsigned)(b.n_pings < 4096 ? b.n_pings : 4096)), dim3(256), 0,
                           s, b.desc, b.n_pings);
    return hipGetLastError();
}

static hipError_t batch_dispatch(const BatchLaunch &b, hipStream_t s, bool query, int *occ)
{
#define SONAR_BK(D, AR)                                           \
    switch (b.K) {                                                \
        case 1: return batch_go<D, 1, AR>(b, s, query, occ);      \
        case 2: return batch_go<D, 2, AR>(b, s, query, occ);      \
        case 3: return batch_go<D, 3, AR>(b, s, query, occ);      \
        default: return batch_go<D, 4, AR>(b, s, query, occ);     \
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
