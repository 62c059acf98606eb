// One ping of the volumetric sonar model, fused in a single kernel.
//
// Per lane (one ray): ray generation in FP64 (Sec. III grid, stratified
// jitter) -> for each bounce: FP32 nearest-hit traversal of the BVH with an
// LDS stack -> FP64 re-intersection of the winner -> scattering, spreading,
// absorption and phase (Sec. II-B) -> for later bounces a connection ray to
// the sensor with an any-hit visibility query -> mirror continuation.
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

// LDS words per wave used by the accumulation stage (bins, values, index).
constexpr int ACC_BIN_WORDS = MAX_BOUNCES * WAVE;             // int bin per slot
constexpr int ACC_VAL_WORDS = MAX_BOUNCES * WAVE * 4;         // float4 per slot
constexpr int ACC_IDX_BASE = ACC_BIN_WORDS + ACC_VAL_WORDS;   // uint16 column index

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

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output number n of the
// generator seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix64_nth(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Triangle record -> vertices, id bits.
struct TriF {
    float3 v0, v1, v2;
    uint32_t idbits;
    float rho, phi;
};
__device__ __forceinline__ TriF load_tri(const float4 *__restrict__ tris, uint32_t i)
{
    float4 a = tris[3 * (size_t)i], b = tris[3 * (size_t)i + 1], c = tris[3 * (size_t)i + 2];
    TriF t;
    t.v0 = make_float3(a.x, a.y, a.z);
    t.v1 = make_float3(a.w, b.x, b.y);
    t.v2 = make_float3(b.z, b.w, c.x);
    t.idbits = __float_as_uint(c.y);
    t.rho = c.z;
    t.phi = c.w;
    return t;
}

struct Ray32 {
    float3 o, d, inv;
};

__device__ __forceinline__ Ray32 make_ray32(d3 o, d3 d)
{
    Ray32 r;
    r.o = f3(o);
    r.d = f3(d);
    // zero components get a tiny signed value so that slab distances stay finite or infinite, never NaN
    float dx = fabsf(r.d.x) > 1e-30f ? r.d.x : copysignf(1e-30f, r.d.x);
    float dy = fabsf(r.d.y) > 1e-30f ? r.d.y : copysignf(1e-30f, r.d.y);
    float dz = fabsf(r.d.z) > 1e-30f ? r.d.z : copysignf(1e-30f, r.d.z);
    r.inv = make_float3(1.0f / dx, 1.0f / dy, 1.0f / dz);
    return r;
}

// Slab test of one box against [tmin, tmax]; the far distance is widened by
// 5e-7 relative so that FP32 rounding never rejects a box the exact ray meets.
__device__ __forceinline__ bool slab(const Ray32 &r, float lx, float ly, float lz, float hx, float hy, float hz,
                                     float tmin, float tmax, float &tnear)
{
    float x0 = (lx - r.o.x) * r.inv.x, x1 = (hx - r.o.x) * r.inv.x;
    float y0 = (ly - r.o.y) * r.inv.y, y1 = (hy - r.o.y) * r.inv.y;
    float z0 = (lz - r.o.z) * r.inv.z, z1 = (hz - r.o.z) * r.inv.z;
    float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), tmin));
    float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tmax));
    tnear = tn;
    return tn <= tf * 1.0000005f;
}

// FP32 Moller-Trumbore (closed triangle). Returns t or -1.
__device__ __forceinline__ float mt32(const Ray32 &r, const TriF &t)
{
    float3 e1 = fsub(t.v1, t.v0), e2 = fsub(t.v2, t.v0);
    float3 p = fcross(r.d, e2);
    float det = fdot(e1, p);
    if (det == 0.f) return -1.f;
    float inv = 1.0f / det;
    float3 tv = fsub(r.o, t.v0);
    float u = fdot(tv, p) * inv;
    if (!(u >= 0.f && u <= 1.f)) return -1.f;
    float3 q = fcross(tv, e1);
    float v = fdot(r.d, q) * inv;
    if (!(v >= 0.f && u + v <= 1.f)) return -1.f;
    return fdot(e2, q) * inv;
}

// Stack-based BVH traversal (near child first). ANY = true returns at the
// first valid hit. `skip` is an original triangle index never reported.
// Returns the triangle record index, or -1; `overflow` is set when the LDS
// stack of DEPTH entries would overflow (the ray is then reported as a miss).
template <int DEPTH, bool ANY>
__device__ int traverse(const float4 *__restrict__ nodes, const float4 *__restrict__ tris, const Ray32 &r,
                        float tmin, float tmax, uint32_t skip, uint32_t *__restrict__ stk, int lane, bool &overflow,
                        float &t_out, uint32_t max_steps)
{
    int best = -1;
    float best_t = tmax;
    uint32_t best_id = 0xFFFFFFFFu;
    uint32_t cur = 0;
    int sp = 0;
    for (uint32_t step = 0;; ++step) {
        if (step >= max_steps) {   // bound on node visits: every wave exits
            overflow = true;
            best = -1;
            break;
        }
        if (!(cur & LEAF_BIT)) {
            const float4 *n = nodes + 4 * (size_t)cur;
            float4 a = n[0], b = n[1], c = n[2], d = n[3];
            float t0, t1;
            bool h0 = slab(r, a.x, a.y, a.z, a.w, b.x, b.y, tmin, best_t, t0);
            bool h1 = slab(r, b.z, b.w, c.x, c.y, c.z, c.w, tmin, best_t, t1);
            uint32_t l0 = __float_as_uint(d.x), l1 = __float_as_uint(d.y);
            if (h0 && h1) {
                uint32_t nearc = t0 <= t1 ? l0 : l1;
                uint32_t farc = t0 <= t1 ? l1 : l0;
                if (sp >= DEPTH) {
                    overflow = true;
                    best = -1;
                    break;
                }
                stk[sp * WAVE + lane] = farc;
                ++sp;
                cur = nearc;
                continue;
            } else if (h0) {
                cur = l0;
                continue;
            } else if (h1) {
                cur = l1;
                continue;
            }
        } else if (cur != EMPTY_LINK) {
            uint32_t first = (cur & 0x7FFFFFFFu) >> 3;
            uint32_t cnt = (cur & 7u) + 1u;
            for (uint32_t k = 0; k < cnt; ++k) {
                TriF t = load_tri(tris, first + k);
                uint32_t id = t.idbits & 0x7FFFFFFFu;
                if (id == skip) continue;
                float th = mt32(r, t);
                if (th > tmin && (th < best_t || (th == best_t && id < best_id))) {
                    best = (int)(first + k);
                    best_t = th;
                    best_id = id;
                    if (ANY) break;
                }
            }
            if (ANY && best >= 0) break;
        }
        if (sp == 0) break;
        --sp;
        cur = stk[sp * WAVE + lane];
    }
    t_out = best_t;
    return best;
}

// FP64 re-intersection of a triangle record (Moller-Trumbore in FP64).
__device__ __forceinline__ double refine64(const TriF &t, d3 o, d3 d, d3 &nrm)
{
    d3 v0 = mk3(t.v0.x, t.v0.y, t.v0.z), v1 = mk3(t.v1.x, t.v1.y, t.v1.z), v2 = mk3(t.v2.x, t.v2.y, t.v2.z);
    d3 e1 = v1 - v0, e2 = v2 - v0;
    d3 p = cross3(d, e2);
    double det = dot3(e1, p);
    d3 tv = o - v0;
    d3 q = cross3(tv, e1);
    double th = dot3(e2, q) / det;
    d3 n = cross3(e1, e2);
    nrm = n * (1.0 / sqrt(dot3(n, n)));
    return th;
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

}  // namespace

template <int DEPTH, int K>
__global__ __launch_bounds__(BLOCK) void k_ping(PingArgs a, int wave_words)
{
    extern __shared__ uint32_t lds[];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    uint32_t *W = lds + (size_t)wave * wave_words;

    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t gid = (int64_t)tile * BLOCK + threadIdx.x;
    const int64_t beam = gid >> a.log2_nr;
    const int j = (int)(gid & (a.n_r - 1));
    const bool active = beam < a.n_beams;

    Slot slot[MAX_BOUNCES];
#pragma unroll
    for (int k = 0; k < MAX_BOUNCES; ++k) slot[k] = Slot{-1, 0.f, 0.f, 0.f};
    float gfeat[7] = {0, 0, 0, 0, 0, 0, 0};
    bool overflow = false;

    if (active) {
        // ---- ray generation (FP64)
        const int h = (int)(beam % a.beams_h), v = (int)(beam / a.beams_h);
        double az, el;
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

#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s_lim = (K == 1) ? a.r_max : 2.0 * a.r_max - L_out;
            int rec_tri = -1, rec_vis = 0;
            if (s_lim > EPS_SELF) {
                Ray32 r = make_ray32(o, d);
                float tf;
                int ti = traverse<DEPTH, false>(a.nodes, a.tris, r, (float)EPS_SELF,
                                                (float)(s_lim * (1.0 + 1e-6)), prev, W, lane, overflow, tf,
                                                a.max_steps);
                if (ti >= 0) {
                    TriF tr = load_tri(a.tris, (uint32_t)ti);
                    d3 nh;
                    double s = refine64(tr, o, d, nh);
                    if (s > EPS_SELF && s <= s_lim) {
                        uint32_t id = tr.idbits & 0x7FFFFFFFu;
                        rec_tri = (int)id;
                        d3 X = o + d * s;
                        L_out += s;
                        T_out += s / a.c0;
                        double dn = dot3(nh, d);
                        d3 np = dn > 0.0 ? nh * -1.0 : nh;
                        double cos_i = -dot3(np, d);
                        d3 rh = d - np * (2.0 * dot3(np, d));
                        const bool pr = (tr.idbits & MAT_BIT) != 0;
                        double rho = pr ? 1.0 : (double)tr.rho;
                        double kd = pr ? 0.0 : a.k_d;
                        double ks = pr ? 1.0 : a.k_s;
                        double phi = pr ? 0.0 : (double)tr.phi;
                        double sgn = pr ? -1.0 : 1.0;

                        double L_back, T_back;
                        d3 w;
                        bool vis = true;
                        if (k == 0) {
                            L_back = L_out;
                            T_back = T_out;
                            w = d * -1.0;
                        } else {
                            d3 toS = S - X;
                            L_back = sqrt(dot3(toS, toS));
                            w = toS * (1.0 / L_back);
                            T_back = L_back / a.c0;
                            // arrival direction (from S toward P) inside the field of view
                            d3 av = w * -1.0;
                            double sx = a.rot[0] * av.x + a.rot[3] * av.y + a.rot[6] * av.z;
                            double sy = a.rot[1] * av.x + a.rot[4] * av.y + a.rot[7] * av.z;
                            double sz = a.rot[2] * av.x + a.rot[5] * av.y + a.rot[8] * av.z;
                            double aza = atan2(sy, sx), ela = atan2(sz, sqrt(sx * sx + sy * sy));
                            if (fabs(aza) > 0.5 * a.hfov || fabs(ela) > 0.5 * a.vfov) vis = false;
                            if (vis && L_back > 2.0 * EPS_SELF) {
                                Ray32 cr = make_ray32(X, w);
                                float ta;
                                int hb = traverse<DEPTH, true>(a.nodes, a.tris, cr, (float)EPS_SELF,
                                                               (float)(L_back - EPS_SELF), id, W, lane, overflow,
                                                               ta, a.max_steps);
                                if (hb >= 0) vis = false;
                            }
                        }
                        rec_vis = vis ? 1 : 0;
                        if (vis) {
                            double cos_o = dot3(np, w);
                            if (cos_o > 0.0) {
                                double Tt = T_out + T_back;
                                double reff = a.c_ref * Tt / 2.0;
                                double x = (reff - a.r_min) / a.dr;
                                double fb = floor(x);
                                if (fb >= 0.0 && fb < (double)a.n_bins) {
                                    double lobe = dot3(rh, w);
                                    lobe = lobe > 0.0 ? lobe : 0.0;
                                    double spec = ks != 0.0 ? ks * pow(lobe, a.phong_n) : 0.0;
                                    double fsc = rho * (kd * cos_i * cos_o + spec);
                                    double amp = Wt * sgn * sqrt(fsc) *
                                                 exp(-a.alpha_db * (L_out + L_back) * LN10_OVER_20) /
                                                 (L_out * L_back * a.n_r);
                                    double cyc = a.f0 * Tt;
                                    double ph = TWO_PI * (cyc - floor(cyc)) + phi;
                                    ph -= TWO_PI * rint(ph / TWO_PI);
                                    float sn, cs;
                                    sincosf((float)ph, &sn, &cs);
                                    slot[k].bin = (int)fb;
                                    slot[k].re = (float)amp * cs;
                                    slot[k].im = (float)amp * sn;
                                    slot[k].inc = (float)(amp * amp);
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
                        }
                        // continuation
                        if (k + 1 < K) {
                            Wt *= sqrt(rho * ks) * sgn;
                            d3 xs = X - S;
                            double lb = (L_out + sqrt(dot3(xs, xs))) / 2.0;
                            if (Wt == 0.0 || lb >= a.r_max) {
                                s_lim = -1.0;   // stop
                            }
                            o = X;
                            d = rh;
                            prev = id;
                        }
                    }
                }
            }
            if (a.rec_tri) {
                size_t ri = ray * K + k;
                a.rec_tri[ri] = rec_tri;
                a.rec_bin[ri] = slot[k].bin;
                a.rec_vis[ri] = rec_vis;
                a.rec_amp[ri] = make_float2(slot[k].re, slot[k].im);
            }
            if (rec_tri < 0 || s_lim < 0.0) {
                for (int q = k + 1; q < K; ++q) {
                    if (a.rec_tri) {
                        size_t ri = ray * K + q;
                        a.rec_tri[ri] = -1;
                        a.rec_bin[ri] = -1;
                        a.rec_vis[ri] = 0;
                        a.rec_amp[ri] = make_float2(0.f, 0.f);
                    }
                }
                break;
            }
        }
        if (masked) {
#pragma unroll
            for (int k = 0; k < MAX_BOUNCES; ++k) slot[k].bin = -1;
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
            float4 *g = reinterpret_cast<float4 *>(a.gbuf + (size_t)beam * 8);
            g[0] = make_float4(gfeat[0] * inv, gfeat[1] * inv, gfeat[2] * inv, gfeat[3] * inv);
            g[1] = make_float4(gfeat[4] * inv, gfeat[5] * inv, cnt / a.n_r, 0.f);
        }
    }

    // ---- accumulation: fixed-order reduction of equal (beam, bin) slots
    wave_sync();
    int *sbin = reinterpret_cast<int *>(W);
    float4 *sval = reinterpret_cast<float4 *>(W + ACC_BIN_WORDS);
    uint16_t *sidx = reinterpret_cast<uint16_t *>(W + ACC_IDX_BASE);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        sbin[k * WAVE + lane] = slot[k].bin;
        sval[k * WAVE + lane] = k == 0 ? make_float4(slot[k].re, slot[k].im, slot[k].inc, 0.f)
                                       : make_float4(slot[k].re, slot[k].im, 0.f, slot[k].inc);
    }
    wave_sync();
    const int nr = a.n_r;
    const int bl = lane >> a.log2_nr;          // beam within the wave
    const int base_lane = bl << a.log2_nr;
    bool head[MAX_BOUNCES];
    float4 sum[MAX_BOUNCES];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        head[k] = false;
        sum[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        int mb = slot[k].bin;
        if (mb < 0) continue;
        int me = j * K + k;
        bool hd = true;
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int jj = 0; jj < nr; ++jj) {
            for (int kk = 0; kk < K; ++kk) {
                int s2 = kk * WAVE + base_lane + jj;
                if (sbin[s2] != mb) continue;
                int o2 = jj * K + kk;
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
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (head[k]) sval[k * WAVE + lane] = sum[k];

    const int bpw = WAVE >> a.log2_nr;
    const int64_t wave_beam0 = (((int64_t)tile * BLOCK) + wave * WAVE) >> a.log2_nr;
    const int nb = a.n_bins;
    const int idx_words = (nb + 1) / 2;
    uint32_t *sidx32 = W + ACC_IDX_BASE;
    for (int q = 0; q < bpw; ++q) {
        const int64_t gb = wave_beam0 + q;
        if (gb >= a.n_beams) break;
        for (int w = lane; w < idx_words; w += WAVE) sidx32[w] = 0u;
        wave_sync();
        if (bl == q) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (head[k]) sidx[slot[k].bin] = (uint16_t)(k * WAVE + lane + 1);
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
                reinterpret_cast<float4 *>(col)[w] = make_float4(v0.x, v0.y, v1.x, v1.y);
                if (i1) {
                    reinterpret_cast<float2 *>(i1)[w] = make_float2(v0.z, v1.z);
                    reinterpret_cast<float2 *>(im)[w] = make_float2(v0.w, v1.w);
                }
            }
        } else {
            for (int b = lane; b < nb; b += WAVE) {
                uint32_t s0 = sidx[b];
                float4 v0 = s0 ? sval[s0 - 1] : make_float4(0.f, 0.f, 0.f, 0.f);
                col[b] = make_float2(v0.x, v0.y);
                if (i1) {
                    i1[b] = v0.z;
                    im[b] = v0.w;
                }
            }
        }
        if (a.det_count) {
            // CA-CFAR on the column while it is still indexed in LDS. A bin
            // without a return has power N0 <= the training mean, and alpha(N)
            // > 1, so only bins holding a return can be detected; the training
            // sums are N * N0 plus the returns inside each window.
            const float n0 = a.det_n0;
            uint64_t key[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                key[k] = 0ull;
                if (bl != q || !head[k]) continue;
                const int bin = slot[k].bin;
                const float4 v = sum[k];
                const float p = v.x * v.x + v.y * v.y + n0;
                float pl = n0, pr = n0;
                if (bin > 0) {
                    uint32_t sl = sidx[bin - 1];
                    if (sl) { float4 u = sval[sl - 1]; pl = u.x * u.x + u.y * u.y + n0; }
                }
                if (bin + 1 < nb) {
                    uint32_t sr = sidx[bin + 1];
                    if (sr) { float4 u = sval[sr - 1]; pr = u.x * u.x + u.y * u.y + n0; }
                }
                if ((bin > 0 && !(p > pl)) || (bin + 1 < nb && !(p >= pr))) continue;
                const int l0 = max(bin - a.det_G - a.det_T, 0), l1 = max(bin - a.det_G, 0);
                const int h0 = min(bin + a.det_G + 1, nb), h1 = min(bin + a.det_G + a.det_T + 1, nb);
                const int N = (l1 - l0) + (h1 - h0);
                if (N <= 0) continue;
                double wsum = (double)N * (double)n0;
                for (int side = 0; side < 2; ++side) {
                    const int p0 = side ? h0 : l0, p1 = side ? h1 : l1;
                    for (int pos = p0; pos < p1; ++pos) {
                        uint32_t sz = sidx[pos];
                        if (sz) {
                            float4 u = sval[sz - 1];
                            float pz = u.x * u.x + u.y * u.y + n0;
                            wsum += (double)pz - (double)n0;
                        }
                    }
                }
                const double thr = a.det_alpha[N] * wsum / N;
                if ((double)p > thr) key[k] = ((uint64_t)__float_as_uint(p) << 32) | (uint32_t)(~bin);
            }
            // the det_M strongest over the beam's lanes, strongest first
            unsigned taken = 0u;
            int cnt = 0;
            for (int m = 0; m < a.det_M; ++m) {
                uint64_t my = 0ull;
                int myk = -1;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (!((taken >> k) & 1u) && key[k] > my) { my = key[k]; myk = k; }
                uint64_t best = my;
                for (int off = 1; off < nr; off <<= 1) {
                    uint64_t o = __shfl_xor(best, off);
                    best = o > best ? o : best;
                }
                if (best == 0ull) break;
                if (myk >= 0 && my == best) taken |= 1u << myk;
                if (j == 0) {
                    a.det_bins[(size_t)gb * a.det_M + m] = (int)(~(uint32_t)(best & 0xFFFFFFFFu));
                    a.det_pw[(size_t)gb * a.det_M + m] = __uint_as_float((uint32_t)(best >> 32));
                }
                cnt = m + 1;
            }
            if (bl == q && j == 0) a.det_count[gb] = cnt;
        }
        wave_sync();
    }
}

int ping_wave_words(int depth, int n_bins)
{
    int acc = ACC_IDX_BASE + (n_bins + 1) / 2;
    int stk = depth * WAVE;
    return acc > stk ? acc : stk;
}

hipError_t launch_ping(const PingArgs &a, int stack_depth, hipStream_t s)
{
    int64_t threads = (int64_t)a.n_beams * a.n_r;
    int nblocks = (int)((threads + BLOCK - 1) / BLOCK);
    if (nblocks == 0) return hipSuccess;
    int depth = stack_depth <= 32 ? 32 : 64;
    int ww = ping_wave_words(depth, a.n_bins);
    size_t shmem = (size_t)ww * 4 * WAVES_PER_BLOCK;
#define SONAR_LAUNCH(D, KK) hipLaunchKernelGGL((k_ping<D, KK>), dim3(nblocks), dim3(BLOCK), shmem, s, a, ww)
    if (depth == 32) {
        switch (a.K) {
            case 1: SONAR_LAUNCH(32, 1); break;
            case 2: SONAR_LAUNCH(32, 2); break;
            case 3: SONAR_LAUNCH(32, 3); break;
            default: SONAR_LAUNCH(32, 4); break;
        }
    } else {
        switch (a.K) {
            case 1: SONAR_LAUNCH(64, 1); break;
            case 2: SONAR_LAUNCH(64, 2); break;
            case 3: SONAR_LAUNCH(64, 3); break;
            default: SONAR_LAUNCH(64, 4); break;
        }
    }
#undef SONAR_LAUNCH
    return hipGetLastError();
}

}  // namespace sonar
