// Multi-bounce ping in stages, for straight rays and one linear sound-speed
// gradient (Sec. II-B: a bounded number of secondary reflections; Sec. II-A:
// rays curved by Snell's law).
//
// The single fused kernel holds a ray's whole path (up to K nearest-hit and
// K - 1 visibility traversals, FP64 state, every contribution) in one lane:
// its register demand limits it to three waves per SIMD and spills, and
// every wave lasts as long as its slowest ray. Here the work is split by
// kind and handed between kernels through HBM (FP64 ray state, FP32
// traversal queries, winners and contribution slots):
//   generation: the launch queries of bounce 0 (FP32 segments);
//   traversal: one lane per query, the rays of a beam in adjacent lanes;
//             only the FP32 query and the traversal state are live;
//   shading k: FP64 re-intersection of each winner, the return path (the
//             reversed incident path at bounce 0, the connection to the
//             sensor after it), scattering, spreading, absorption, phase,
//             retro-chain returns, the continuation; it writes the ray's
//             record and contribution slot, the next bounce's query and the
//             return path's visibility query;
//   visibility k: the same traversal, any hit: a blocked return path loses
//             its contribution;
//   accumulation: per wave, the rays' contribution slots (masked rays and
//             moved receive-binning returns taken out) reduced in the same
//             fixed order as the fused kernel, with the fused CFAR test and
//             one column write.
// Each ray is traced with the same arithmetic as in the fused kernel, so
// records are identical to it and volumes equal up to FP32 rounding.
#include <hip/hip_runtime.h>
#include <math.h>

#include "trace.hpp"

namespace sonar {

namespace {

// LDS stack entries per lane of the traversal stages (deeper entries go to
// private memory; the multipath scene's deepest traversal needs 14)
constexpr int STG_LDS_STACK = 20;

__device__ __forceinline__ bool ray_masked(const PingArgs &a, size_t ray)
{
    return a.mask && ((a.mask[ray >> 5] >> (ray & 31)) & 1u);
}

// The launch direction of ray j of beam `beam` (FP64, world frame) and the
// transmit pattern there.
__device__ __forceinline__ d3 launch_dir(const PingArgs &a, int64_t beam, int j, float &w_tx)
{
    const int h = (int)(beam % a.beams_h), v = (int)(beam / a.beams_h);
    double az, el;
    w_tx = 1.f;
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
            const float fa = (float)((ja + u1) / a.na - 0.5), fe = (float)((je + u2) / a.ne - 0.5);
            w_tx = exp2f(-2.f * (fa * fa + fe * fe));
        }
    }
    double ce = cos(el), se = sin(el), ca = cos(az), sa = sin(az);
    d3 ds = mk3(ce * ca, ce * sa, se);
    return mk3(a.rot[0] * ds.x + a.rot[1] * ds.y + a.rot[2] * ds.z, a.rot[3] * ds.x + a.rot[4] * ds.y + a.rot[5] * ds.z,
               a.rot[6] * ds.x + a.rot[7] * ds.y + a.rot[8] * ds.z);
}

// Where bounce k starts: the sensor and the launch direction (bounce 0) or
// the state the previous bounce left. Returns false for a stopped ray.
template <bool FIRST>
__device__ __forceinline__ bool bounce_start(const PingArgs &a, size_t ray, int64_t beam, int j, d3 &o, d3 &d,
                                             double &L_out, double &T_out, double &Wt, uint32_t &prev, float &w_tx)
{
    if (FIRST) {
        d = launch_dir(a, beam, j, w_tx);
        o = mk3(a.pos[0], a.pos[1], a.pos[2]);
        L_out = T_out = 0.0;
        Wt = 1.0;
        prev = 0xFFFFFFFFu;
        return true;
    }
    const RayState s = a.stg_state[ray];
    o = mk3(s.o[0], s.o[1], s.o[2]);
    d = mk3(s.d[0], s.d[1], s.d[2]);
    L_out = s.L_out;
    T_out = s.T_out;
    Wt = s.Wt;
    prev = s.prev;
    w_tx = s.w_tx;
    return L_out >= 0.0;
}

// Segment limit of bounce k: arc length for constant c, travel time in a
// gradient (s_lim then bounds the arc length through the fastest speed).
template <bool ARC>
__device__ __forceinline__ double bounce_limit(const PingArgs &a, double L_out, double T_out, double &T_lim)
{
    T_lim = 0.0;
    if (!ARC) return (a.K == 1) ? a.r_max : 2.0 * a.r_max - L_out;
    T_lim = (a.K == 1) ? a.r_max / a.c_ref : 2.0 * a.r_max / a.c_ref - T_out;
    return a.c_hi * T_lim;
}

__device__ __forceinline__ SegRec seg_rec(const Path64 &p, double smin, double smax, uint32_t skip)
{
    const Seg32 g = make_seg(p, smin, smax);
    SegRec r;
    r.o[0] = g.o.x; r.o[1] = g.o.y; r.o[2] = g.o.z; r.sigma = g.sigma;
    r.d[0] = g.d.x; r.d[1] = g.d.y; r.d[2] = g.d.z; r.tmin = g.tmin;
    r.ad[0] = g.ad.x; r.ad[1] = g.ad.y; r.ad[2] = g.ad.z; r.tmax = g.tmax;
    r.anc[0] = g.anc.x; r.anc[1] = g.anc.y; r.anc[2] = g.anc.z; r.kappa = g.kappa;
    r.smin = g.smin;
    r.smax = g.smax;
    r.skip = skip;
    r.live = 1;
    return r;
}

__device__ __forceinline__ Seg32 seg_of(const SegRec &r)
{
    Seg32 g;
    g.o = make_float3(r.o[0], r.o[1], r.o[2]);
    g.d = make_float3(r.d[0], r.d[1], r.d[2]);
    g.inv = safe_inv(g.d);
    g.sigma = r.sigma;
    g.tmin = r.tmin;
    g.tmax = r.tmax;
    g.smin = r.smin;
    g.smax = r.smax;
    g.ad = make_float3(r.ad[0], r.ad[1], r.ad[2]);
    g.anc = make_float3(r.anc[0], r.anc[1], r.anc[2]);
    g.kappa = r.kappa;
    return g;
}

// Launch queries of bounce 0 for every ray.
template <bool ARC>
__global__ __launch_bounds__(256) void k_stage_gen(PingArgs a)
{
    const int64_t gid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (gid >= a.n_rays) return;
    d3 o, d;
    double L_out, T_out, Wt;
    uint32_t prev;
    float w_tx;
    bounce_start<true>(a, (size_t)gid, gid >> a.log2_nr, (int)(gid & (a.n_r - 1)), o, d, L_out, T_out, Wt, prev,
                       w_tx);
    double T_lim;
    const double s_lim = bounce_limit<ARC>(a, L_out, T_out, T_lim);
    SegRec r;
    r.live = 0;
    if (s_lim > EPS_SELF) {
        const Path64 path = ARC ? make_path(o, d, a.g, a.c0) : Path64{o, d, mk3(0, 0, 0), 0.0, false};
        r = seg_rec(path, EPS_SELF, s_lim * (1.0 + 1e-6), prev);
    }
    a.stg_seg[gid] = r;
}

// Traversal of one set of queries (one per ray, one lane each, the rays of
// a beam in adjacent lanes): nearest hit (ANY = false: the winner's record
// index and FP32 arc length go to stg_hit) or any hit (ANY = true: a blocked
// return path of bounce k loses its contribution). Only the FP32 query and
// the traversal state are live.
template <int DEPTH, bool ARC, bool ANY>
__global__ __attribute__((amdgpu_flat_work_group_size(1, 256), amdgpu_waves_per_eu(ARC ? 6 : 8)))
void k_stage_trav(PingArgs a, int k, int wave_words)
{
    extern __shared__ uint32_t lds[];
    uint32_t *W = lds + (size_t)(threadIdx.x / WAVE) * wave_words;
    constexpr int DL = DEPTH > STG_LDS_STACK ? STG_LDS_STACK : DEPTH;
    const int lane = threadIdx.x & (WAVE - 1);
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t gid = (int64_t)tile * BLOCK + threadIdx.x;
    bool overflow = false;
    uint32_t st_nodes = 0, st_tris = 0, st_deep = 0;
    if (gid < a.n_rays) {
        const size_t ray = (size_t)gid;
        const SegRec rec = (ANY ? a.stg_cseg : a.stg_seg)[ray];
        int ti = -1;
        float sf = 0.f;
        if (rec.live)
            ti = traverse<DEPTH, DL, ANY, ARC, false>(as_global(a.nodes), as_global(a.tris), seg_of(rec), rec.skip, W,
                                                      lane, overflow, sf, a.max_steps, st_nodes, st_tris, st_deep);
        if (!ANY) {
            a.stg_hit[ray] = make_int2(ti, __float_as_int(sf));
        } else if (ti >= 0) {
            const size_t sk = (size_t)k * a.n_rays + ray;
            a.stg_bin[sk] = -1;
            a.stg_val[sk] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (a.rec_tri) {
                const size_t ri = ray * a.K + k;
                a.rec_bin[ri] = -1;
                a.rec_vis[ri] = 0;
                a.rec_amp[ri] = make_float2(0.f, 0.f);
            }
        }
    }
    if (overflow) atomicOr(a.status, ST_STACK);
}

// Shading of bounce k for every ray (no traversal): FP64 re-intersection of
// the winner, the return path (the reversed incident path at bounce 0, the
// connection to the sensor after it, whose visibility is left to the next
// stage), scattering, spreading, absorption and phase, retro-chain returns,
// the continuation, the ray's record and contribution slots, and at bounce
// 0 the G-buffer.
template <bool ARC, bool FIRST>
__global__ __launch_bounds__(256) void k_stage_shade(PingArgs a, int k)
{
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t gid = (int64_t)tile * BLOCK + threadIdx.x;
    const int64_t beam = gid >> a.log2_nr;
    const int j = (int)(gid & (a.n_r - 1));
    const bool active = gid < a.n_rays;
    const size_t ray = (size_t)gid;
    const int K = a.K;
    const bool retro = (a.flags & FLAG_RETRO_CHAIN) != 0;
    float gfeat[7] = {0, 0, 0, 0, 0, 0, 0};

    if (active) {
        const d3 S = mk3(a.pos[0], a.pos[1], a.pos[2]);
        d3 o, d;
        double L_out, T_out, Wt;
        uint32_t prev;
        float w_tx;
        const bool stop = !bounce_start<FIRST>(a, ray, beam, j, o, d, L_out, T_out, Wt, prev, w_tx);
        int rec_tri = -1, rec_vis = 0, cbin = -1;
        float cre = 0.f, cim = 0.f, cinc = 0.f;
        float w_rx = w_tx;
        int rxb = (int)beam;
        int rbin = -1;
        float rre = 0.f, rim = 0.f, rinc = 0.f;
        SegRec cq;           // the return path's visibility query (bounce k > 0)
        cq.live = 0;
        SegRec nq;           // the next bounce's nearest-hit query
        nq.live = 0;
        RayState nx;
        nx.L_out = -1.0;     // stopped unless the continuation below says otherwise
        const int2 hit = a.stg_hit[ray];
        const int ti = hit.x;
        if (!stop && ti >= 0) {
            double T_lim;
            const double s_lim = bounce_limit<ARC>(a, L_out, T_out, T_lim);
            const Path64 path = ARC ? make_path(o, d, a.g, a.c0) : Path64{o, d, mk3(0, 0, 0), 0.0, false};
            const float sf = __int_as_float(hit.y);
            {
                {
                    const TriF tr = load_tri(as_global(a.tris), (uint32_t)ti);
                    d3 nh;
                    const double s = refine64(tr, path, (double)sf, nh);
                    const double tau = ARC ? path_time(path, s, a.g, a.c0) : s / a.c0;
                    if (s > EPS_SELF && (ARC ? tau <= T_lim : s <= s_lim)) {
                        const uint32_t id = tr.idbits & 0x7FFFFFFFu;
                        rec_tri = (int)id;
                        const d3 X = ARC ? path_point(path, s) : o + d * s;
                        const d3 din = ARC ? path_tangent(path, s) : d;
                        L_out += s;
                        T_out += tau;
                        const double dn = dot3(nh, din);
                        const d3 np = dn > 0.0 ? nh * -1.0 : nh;
                        const double cos_i = -dot3(np, din);
                        const d3 rh = din - np * (2.0 * dot3(np, din));
                        const bool pr = (tr.idbits & MAT_BIT) != 0;
                        const double rho = pr ? 1.0 : (double)tr.rho;
                        const double kd = pr ? 0.0 : a.k_d;
                        const double ks = pr ? 1.0 : a.k_s;
                        const double phi = pr ? 0.0 : (double)tr.phi;
                        const double sgn = pr ? -1.0 : 1.0;
                        double L_back, T_back;
                        d3 w;
                        bool vis = true;
                        if (FIRST) {
                            L_back = L_out;
                            T_back = T_out;
                            w = din * -1.0;
                        } else {
                            const Conn cn = connect(X, S, ARC ? a.g : 0.0, a.c0);
                            L_back = cn.L;
                            T_back = cn.T;
                            w = cn.w;
                            const d3 av = cn.arrive * -1.0;
                            const double sx = a.rot[0] * av.x + a.rot[3] * av.y + a.rot[6] * av.z;
                            const double sy = a.rot[1] * av.x + a.rot[4] * av.y + a.rot[7] * av.z;
                            const double sz = a.rot[2] * av.x + a.rot[5] * av.y + a.rot[8] * av.z;
                            const double sxy = sqrt(sx * sx + sy * sy);
                            if (a.hfov < M_PI) {
                                if (!(sx > 0.0 && fabs(sy) <= a.tan_h * sx)) vis = false;
                            } else if (fabs(atan2(sy, sx)) > 0.5 * a.hfov) {
                                vis = false;
                            }
                            if (fabs(sz) > a.tan_v * sxy) vis = false;
                            if (vis && a.flags) {
                                const int h = (int)(beam % a.beams_h), v = (int)(beam / a.beams_h);
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
                        const double cos_o = dot3(np, w);
                        if (vis && cos_o > 0.0) {
                            const double Tt = T_out + T_back;
                            const double reff = a.c_ref * Tt / 2.0;
                            const double fb = floor((reff - a.r_min) / a.dr);
                            if (fb >= 0.0 && fb < (double)a.n_bins) {
                                float lobe = (float)dot3(rh, w);
                                lobe = lobe > 0.f ? lobe : 0.f;
                                const double spec = ks != 0.0 ? ks * (double)powf(lobe, (float)a.phong_n) : 0.0;
                                const double fsc = rho * (kd * cos_i * cos_o + spec);
                                const double att = (double)expf((float)(-a.alpha_db * (L_out + L_back) * LN10_OVER_20));
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
                                if (FIRST) {
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
                        if (!FIRST && retro) {
                            float lobe = (float)(-dot3(rh, din));
                            lobe = lobe > 0.f ? lobe : 0.f;
                            const double spec = ks != 0.0 ? ks * (double)powf(lobe, (float)a.phong_n) : 0.0;
                            const double fsc = rho * (kd * cos_i * cos_i + spec);
                            const double fb = floor((a.c_ref * T_out - a.r_min) / a.dr);
                            if (fb >= 0.0 && fb < (double)a.n_bins) {
                                const double att = (double)expf((float)(-a.alpha_db * 2.0 * L_out * LN10_OVER_20));
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
                        if (k + 1 < K) {
                            d3 dc = rh;
                            if ((a.flags & FLAG_DIFFUSE_BOUNCE) && !pr) {
                                Wt *= sqrt(rho * (kd + ks)) * sgn;
                                if (Wt != 0.0) {
                                    const Drawn dw = draw_continuation(a.seed, a.ping, a.phong_n, ray, k, rh, np, kd, ks);
                                    if (!dw.lit) Wt = 0.0;
                                    dc = dw.dir;
                                }
                            } else {
                                Wt *= sqrt(rho * ks) * sgn;
                            }
                            const double dS = norm3(X - S);
                            const double lb = ARC ? a.c_ref * (T_out + dS / a.c_hi) / 2.0 : (L_out + dS) / 2.0;
                            if (!(Wt == 0.0 || lb >= a.r_max)) {
                                nx.o[0] = X.x; nx.o[1] = X.y; nx.o[2] = X.z;
                                nx.d[0] = dc.x; nx.d[1] = dc.y; nx.d[2] = dc.z;
                                nx.L_out = L_out;
                                nx.T_out = T_out;
                                nx.Wt = Wt;
                                nx.prev = id;
                                double T_lim2;
                                const double s_lim2 = bounce_limit<ARC>(a, L_out, T_out, T_lim2);
                                if (s_lim2 > EPS_SELF) {
                                    const Path64 np2 = ARC ? make_path(X, dc, a.g, a.c0)
                                                           : Path64{X, dc, mk3(0, 0, 0), 0.0, false};
                                    nq = seg_rec(np2, EPS_SELF, s_lim2 * (1.0 + 1e-6), id);
                                }
                            }
                        }
                        if (!FIRST && vis && L_back > 2.0 * EPS_SELF) {
                            // the return path is tested for an occluder in the visibility stage
                            const Path64 cp = ARC ? make_path(X, w, a.g, a.c0) : Path64{X, w, mk3(0, 0, 0), 0.0, false};
                            cq = seg_rec(cp, EPS_SELF, L_back - EPS_SELF, id);
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
            const float wr = w_tx * w_tx;
            rre *= wr;
            rim *= wr;
            rinc *= wr * wr;
        }
        if (k + 1 < K) {
            nx.w_tx = w_tx;
            a.stg_state[ray] = nx;
            a.stg_seg[ray] = nq;
        }
        if (!FIRST) a.stg_cseg[ray] = cq;
        const size_t sk = (size_t)k * a.n_rays + ray;
        a.stg_bin[sk] = cbin;
        a.stg_val[sk] = k == 0 ? make_float4(cre, cim, cinc, 0.f) : make_float4(cre, cim, 0.f, cinc);
        if (a.stg_rxb) a.stg_rxb[sk] = rxb;
        if (!FIRST && retro) {
            const size_t sr = (size_t)(K + k - 1) * a.n_rays + ray;
            a.stg_bin[sr] = rbin;
            a.stg_val[sr] = make_float4(rre, rim, 0.f, rinc);
        }
        if (a.rec_tri) {
            const size_t ri = ray * K + k;
            a.rec_tri[ri] = rec_tri;
            a.rec_bin[ri] = cbin;
            a.rec_vis[ri] = rec_vis;
            a.rec_amp[ri] = make_float2(cre, cim);
            if (a.rec_beam) a.rec_beam[ri] = rxb;
            if (retro && a.rec_rbin) {
                a.rec_rbin[ri] = rbin;
                a.rec_ramp[ri] = make_float2(rre, rim);
            }
        }
        if (FIRST && ray_masked(a, ray))
            for (int t = 0; t < 7; ++t) gfeat[t] = 0.f;
    }
    if (FIRST && a.gbuf) {
        // the first-bounce features reduced over the beam's lanes
        for (int off = 1; off < a.n_r; off <<= 1)
            for (int t = 0; t < 7; ++t) gfeat[t] += __shfl_xor(gfeat[t], off);
        if (active && j == 0) {
            const float cnt = gfeat[6];
            const float inv = cnt > 0.f ? 1.f / cnt : 0.f;
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
}

// Accumulation: the wave's 64 rays' KS contribution slots into LDS (masked
// rays and returns that receive binning moves to another beam taken out,
// the latter listed), then the fixed-order reduction and column write.
template <int KS>
__global__ __launch_bounds__(256) void k_stage_accumulate(PingArgs a, int wave_words)
{
    extern __shared__ uint32_t lds[];
    uint32_t *W = lds + (size_t)(threadIdx.x / WAVE) * wave_words;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t gid = (int64_t)tile * BLOCK + threadIdx.x;
    const int64_t beam = gid >> a.log2_nr;
    const int j = (int)(gid & (a.n_r - 1));
    const bool active = gid < a.n_rays;
    const size_t ray = (size_t)gid;
    int *sbin = reinterpret_cast<int *>(W);
    float4 *sval = reinterpret_cast<float4 *>(W + KS * WAVE);
    uint32_t *sidx32 = W + 5 * KS * WAVE;
    const bool masked = active && ray_masked(a, ray);
    const bool rx = a.K > 1 && (a.flags & FLAG_RX_BEAMS);
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        int bin = -1;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (active) {
            const size_t sk = (size_t)k * a.n_rays + ray;
            bin = a.stg_bin[sk];
            v = a.stg_val[sk];
        }
        if (rx && k > 0 && k < a.K) {
            const int rxb = active ? a.stg_rxb[(size_t)k * a.n_rays + ray] : (int)beam;
            const bool away = bin >= 0 && rxb != (int)beam;
            rx_append(a, away && !masked, make_int4(rxb, bin, __float_as_int(v.x), __float_as_int(v.y)), lane);
            if (away) bin = -1;
        }
        if (masked) bin = -1;
        sbin[k * WAVE + lane] = bin;
        sval[k * WAVE + lane] = v;
    }
    wave_sync();
    reduce_tile<KS>(a, (int64_t)tile * BLOCK, wave, lane, j, active, sbin, sval, sidx32);
}

int stage_stack_words(int depth) { return (depth > STG_LDS_STACK ? STG_LDS_STACK : depth) * WAVE; }

}  // namespace

size_t staged_workspace_bytes(int64_t n_rays, int K, bool retro, bool rx)
{
    if (K < 2) return 0;
    const size_t KS = retro ? 2 * (size_t)K - 1 : (size_t)K;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t b = up(sizeof(RayState) * (size_t)n_rays) + 2 * up(sizeof(SegRec) * (size_t)n_rays) +
               up(sizeof(int2) * (size_t)n_rays) +
               up(sizeof(int32_t) * KS * (size_t)n_rays) + up(sizeof(float4) * KS * (size_t)n_rays);
    if (rx) b += up(sizeof(int32_t) * (size_t)K * (size_t)n_rays);
    return b;
}

void set_staged_area(PingArgs &a, void *area)
{
    const bool retro = (a.flags & FLAG_RETRO_CHAIN) != 0;
    const bool rx = (a.flags & FLAG_RX_BEAMS) != 0;
    const size_t n = (size_t)a.n_rays;
    const size_t KS = retro ? 2 * (size_t)a.K - 1 : (size_t)a.K;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *p = reinterpret_cast<char *>(area);
    a.stg_state = reinterpret_cast<RayState *>(p);
    p += up(sizeof(RayState) * n);
    a.stg_seg = reinterpret_cast<SegRec *>(p);
    p += up(sizeof(SegRec) * n);
    a.stg_cseg = reinterpret_cast<SegRec *>(p);
    p += up(sizeof(SegRec) * n);
    a.stg_hit = reinterpret_cast<int2 *>(p);
    p += up(sizeof(int2) * n);
    a.stg_bin = reinterpret_cast<int32_t *>(p);
    p += up(sizeof(int32_t) * KS * n);
    a.stg_val = reinterpret_cast<float4 *>(p);
    p += up(sizeof(float4) * KS * n);
    a.stg_rxb = rx ? reinterpret_cast<int32_t *>(p) : nullptr;

}

template <int DEPTH, bool ARC>
static void stage_sequence(const PingArgs &a, int nblocks, hipStream_t s)
{
    const int ww = stage_stack_words(DEPTH);
    const size_t shmem = (size_t)ww * 4 * WAVES_PER_BLOCK;
    hipLaunchKernelGGL((k_stage_gen<ARC>), dim3(nblocks), dim3(BLOCK), 0, s, a);
    for (int k = 0; k < a.K; ++k) {
        hipLaunchKernelGGL((k_stage_trav<DEPTH, ARC, false>), dim3(nblocks), dim3(BLOCK), shmem, s, a, k, ww);
        if (k == 0) hipLaunchKernelGGL((k_stage_shade<ARC, true>), dim3(nblocks), dim3(BLOCK), 0, s, a, k);
        else hipLaunchKernelGGL((k_stage_shade<ARC, false>), dim3(nblocks), dim3(BLOCK), 0, s, a, k);
        if (k > 0) hipLaunchKernelGGL((k_stage_trav<DEPTH, ARC, true>), dim3(nblocks), dim3(BLOCK), shmem, s, a, k, ww);
    }
}

hipError_t launch_ping_staged(const PingArgs &a, int stack_depth, hipStream_t s)
{
    const int64_t threads = a.n_rays;
    const int nblocks = (int)((threads + BLOCK - 1) / BLOCK);
    if (nblocks == 0) return hipSuccess;
    const bool retro = (a.flags & FLAG_RETRO_CHAIN) != 0;
    const int KS = retro ? 2 * a.K - 1 : a.K;
    const int aww = (5 * KS * WAVE + (a.n_bins + 1) / 2 + 3) & ~3;
    const size_t ashm = (size_t)aww * 4 * WAVES_PER_BLOCK;
    // the accumulation block's LDS (slots and column index) must stay within
    // 64 KB; beyond that (retro-chain returns of four bounces over more than
    // about 3,400 bins) the fused kernel runs instead
    if (ashm > 65536) return launch_ping(a, stack_depth, s);
    const bool arc = a.g != 0.0;
    if (stack_depth > 32) {
        if (arc) stage_sequence<64, true>(a, nblocks, s);
        else stage_sequence<64, false>(a, nblocks, s);
    } else {
        if (arc) stage_sequence<32, true>(a, nblocks, s);
        else stage_sequence<32, false>(a, nblocks, s);
    }
    switch (KS) {
        case 2: hipLaunchKernelGGL((k_stage_accumulate<2>), dim3(nblocks), dim3(BLOCK), ashm, s, a, aww); break;
        case 3: hipLaunchKernelGGL((k_stage_accumulate<3>), dim3(nblocks), dim3(BLOCK), ashm, s, a, aww); break;
        case 4: hipLaunchKernelGGL((k_stage_accumulate<4>), dim3(nblocks), dim3(BLOCK), ashm, s, a, aww); break;
        case 5: hipLaunchKernelGGL((k_stage_accumulate<5>), dim3(nblocks), dim3(BLOCK), ashm, s, a, aww); break;
        default: hipLaunchKernelGGL((k_stage_accumulate<7>), dim3(nblocks), dim3(BLOCK), ashm, s, a, aww); break;
    }
    return hipGetLastError();
}

}  // namespace sonar
