// Host side of the C-ABI: validation, scene ownership and launches.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "internal.hpp"
#include "surrogate.hpp"

#include <stdlib.h>

#include <mutex>
#include <string>
#include <vector>

struct sonar_scene {
    sonar::Scene s;
};

struct sonar_surrogate {
    sonar::Surrogate *s = nullptr;
};

struct sonar_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

thread_local char g_err[512] = "";

sonar_status fail(sonar_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int x)
{
    int l = 0;
    while ((1 << (l + 1)) <= x) ++l;
    return l;
}

void free_scene_mem(sonar::Scene &s)
{
    if (s.nodes) (void)hipFree(s.nodes);
    if (s.tris) (void)hipFree(s.tris);
    if (s.status) (void)hipFree(s.status);
    s.nodes = nullptr;
    s.tris = nullptr;
    s.status = nullptr;
}

sonar_status check_params(const sonar_params *p)
{
    if (!p) return fail(SONAR_E_INVALID, "params is NULL");
    if (!(p->hfov > 0 && p->hfov < 2 * M_PI) || !(p->vfov > 0 && p->vfov < M_PI))
        return fail(SONAR_E_INVALID, "fields of view must satisfy 0 < hfov < 2 pi, 0 < vfov < pi");
    if (p->n_h < 1 || p->n_v < 1 || p->n_h > 65536 || p->n_v > 65536)
        return fail(SONAR_E_INVALID, "n_h and n_v must be in [1, 65536]");
    if (!is_pow2(p->rays_per_beam) || p->rays_per_beam > 64)
        return fail(SONAR_E_INVALID, "rays_per_beam must be a power of two in [1, 64]");
    if (p->grid_mode != 0 && p->grid_mode != 1) return fail(SONAR_E_INVALID, "grid_mode must be 0 or 1");
    if (p->grid_mode == 1 && p->rays_per_beam != 1)
        return fail(SONAR_E_INVALID, "the LiDAR firing grid takes one ray per emitter");
    if (p->n_range < 1 || p->n_range > sonar::MAX_BINS)
        return fail(SONAR_E_INVALID, "n_range must be in [1, %d]", sonar::MAX_BINS);
    if (!(p->r_min >= 0) || !(p->r_max > p->r_min) || !isfinite(p->r_max))
        return fail(SONAR_E_INVALID, "need 0 <= r_min < r_max < inf");
    if (!(p->freq_hz > 0) || !isfinite(p->freq_hz)) return fail(SONAR_E_INVALID, "freq_hz must be positive");
    if (!(p->c0 > 0) || !isfinite(p->c0) || !isfinite(p->c_grad)) return fail(SONAR_E_INVALID, "bad sound speed");
    if (!(p->abs_db_per_m >= 0) || !isfinite(p->abs_db_per_m))
        return fail(SONAR_E_INVALID, "abs_db_per_m must be >= 0");
    if (p->max_bounces < 1 || p->max_bounces > sonar::MAX_BOUNCES)
        return fail(SONAR_E_INVALID, "max_bounces must be in [1, %d]", sonar::MAX_BOUNCES);
    if (!(p->k_d >= 0) || !(p->k_s >= 0) || !(p->phong_n >= 0) || !isfinite(p->k_d) || !isfinite(p->k_s) ||
        !isfinite(p->phong_n))
        return fail(SONAR_E_INVALID, "k_d, k_s and phong_n must be finite and >= 0");
    int64_t beams = (int64_t)(p->n_h + (p->grid_mode == 1)) * (p->n_v + (p->grid_mode == 1));
    if (beams * p->rays_per_beam > ((int64_t)1 << 31) - 1) return fail(SONAR_E_INVALID, "too many rays");
    if (p->flags & ~(SONAR_FLAG_BEAM_PATTERN | SONAR_FLAG_RX_BEAMS | SONAR_FLAG_DIFFUSE_BOUNCE | SONAR_FLAG_RETRO_CHAIN))
        return fail(SONAR_E_INVALID, "unknown flags");
    if ((p->flags & (SONAR_FLAG_BEAM_PATTERN | SONAR_FLAG_RX_BEAMS)) && p->grid_mode != 0)
        return fail(SONAR_E_UNSUPPORTED, "beam pattern and receive binning need cell-centred beams (grid_mode 0)");
    return SONAR_OK;
}

sonar_status check_pose(const sonar_pose *q)
{
    if (!q) return fail(SONAR_E_INVALID, "pose is NULL");
    for (int i = 0; i < 3; ++i)
        if (!isfinite(q->position[i])) return fail(SONAR_E_INVALID, "non-finite pose position");
    // rotation: orthonormal within 1e-6
    const double *R = q->rot;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double d = R[i] * R[j] + R[3 + i] * R[3 + j] + R[6 + i] * R[6 + j];
            double want = i == j ? 1.0 : 0.0;
            if (!(fabs(d - want) <= 1e-6)) return fail(SONAR_E_INVALID, "pose rotation is not orthonormal");
        }
    return SONAR_OK;
}

int beams_h_of(const sonar_params *p) { return p->grid_mode == 1 ? p->n_h + 1 : p->n_h; }
int beams_v_of(const sonar_params *p) { return p->grid_mode == 1 ? p->n_v + 1 : p->n_v; }

static_assert(SONAR_FLAG_BEAM_PATTERN == sonar::FLAG_BEAM_PATTERN && SONAR_FLAG_RX_BEAMS == sonar::FLAG_RX_BEAMS &&
                  SONAR_FLAG_DIFFUSE_BOUNCE == sonar::FLAG_DIFFUSE_BOUNCE,
              "beam flags");

// Receive binning with several bounces lists the returns it moves.
static bool needs_rx_list(const sonar_params *p)
{
    return (p->flags & SONAR_FLAG_RX_BEAMS) && p->max_bounces > 1;
}

// Bytes of the receive-binning area: a 256-byte counter block, then one
// 16-byte entry per possible moved return (n_rays * (max_bounces - 1)).
static size_t rx_bytes(const sonar_params *p)
{
    const int64_t rays = (int64_t)beams_h_of(p) * beams_v_of(p) * p->rays_per_beam;
    return 256 + 16 * (size_t)rays * (size_t)(p->max_bounces - 1);
}

static void set_rx_area(sonar::PingArgs &a, const sonar_params *p, void *area)
{
    a.rx_count = reinterpret_cast<uint32_t *>(area);
    a.rx_list = reinterpret_cast<int4 *>(reinterpret_cast<char *>(area) + 256);
    a.rx_cap = (uint32_t)(a.n_rays * (p->max_bounces - 1));
}

// Staged multi-bounce buffers of one ping: 0 for a single bounce (the
// fused kernel always applies then).
static size_t staged_bytes(const sonar_params *p)
{
    if (p->max_bounces < 2) return 0;
    const int64_t rays = (int64_t)beams_h_of(p) * beams_v_of(p) * p->rays_per_beam;
    return sonar::staged_workspace_bytes(rays, p->max_bounces, (p->flags & SONAR_FLAG_RETRO_CHAIN) != 0,
                                         (p->flags & SONAR_FLAG_RX_BEAMS) != 0);
}

// The ping kernels: staged when their area is set, else the fused kernel.
static hipError_t launch_any(const sonar::PingArgs &a, int stack, hipStream_t s)
{
    return a.stg_state ? sonar::launch_ping_staged(a, stack, s) : sonar::launch_ping(a, stack, s);
}

// reset -> ping -> scatter of the moved returns (or the plain ping)
static hipError_t launch_ping_rx(const sonar::PingArgs &a, int stack, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (a.rx_list) e = sonar::launch_rx_reset(a.rx_count, s);
    if (e == hipSuccess) e = launch_any(a, stack, s);
    if (e == hipSuccess && a.rx_list) e = sonar::launch_rx_scatter(a, s);
    return e;
}

sonar_status fill_ping_args(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q, sonar_cf32 *volume,
                            float *gbuffer, float *incoh, const sonar_ray_record *rec, const uint32_t *ray_mask,
                            sonar::PingArgs *out)
{
    if (!sc) return fail(SONAR_E_INVALID, "scene is NULL");
    sonar_status st = check_params(p);
    if (st != SONAR_OK) return st;
    if ((st = check_pose(q)) != SONAR_OK) return st;
    if (!volume) return fail(SONAR_E_INVALID, "volume is NULL");
    if (rec && (!rec->tri || !rec->bin || !rec->vis || !rec->amp))
        return fail(SONAR_E_INVALID, "record arrays tri, bin, vis and amp must all be set");
    if (rec && (!rec->retro_bin) != (!rec->retro_amp))
        return fail(SONAR_E_INVALID, "record arrays retro_bin and retro_amp go together");
    if ((p->flags & SONAR_FLAG_RETRO_CHAIN) && p->max_bounces > 1) {
        if (rec && rec->stats)
            return fail(SONAR_E_UNSUPPORTED, "traversal counters are not kept with retro-chain returns");
        const int max_bins = p->max_bounces == 3 ? 3328 : (p->max_bounces == 4 ? 3584 : 4096);
        if (p->n_range > max_bins)
            return fail(SONAR_E_UNSUPPORTED, "retro-chain returns with %d bounces take at most %d bins",
                        p->max_bounces, max_bins);
    }
    // a sound speed must stay positive over the scene and the sensor
    if (p->c_grad != 0.0) {
        double zmax = fmax((double)sc->s.zabs_max, fabs(q->position[2])) + 1.0;
        if (!(p->c0 - fabs(p->c_grad) * zmax > 0.0))
            return fail(SONAR_E_INVALID, "c(z) = c0 + c_grad z must stay positive over the scene");
        if (fabs(p->c_grad) * 2.0 * p->r_max / (p->c0 - fabs(p->c_grad) * zmax) > 1e-2)
            return fail(SONAR_E_UNSUPPORTED, "ray curvature too strong for one chord per segment (|g| 2 r_max / c > 1e-2)");
    }
    if (sc->s.stack > 64)
        return fail(SONAR_E_STACK, "hierarchy of %d levels can need %d stack entries, more than 64", sc->s.depth,
                    sc->s.stack);
    sonar::PingArgs &a = *out;
    memset(&a, 0, sizeof(a));
    a.nodes = sc->s.nodes;
    a.tris = sc->s.tris;
    a.status = sc->s.status;
    for (int i = 0; i < 3; ++i) a.pos[i] = q->position[i];
    for (int i = 0; i < 9; ++i) a.rot[i] = q->rot[i];
    a.hfov = p->hfov;
    a.vfov = p->vfov;
    a.dth_h = p->hfov / p->n_h;
    a.dth_v = p->vfov / p->n_v;
    a.r_min = p->r_min;
    a.r_max = p->r_max;
    a.dr = (p->r_max - p->r_min) / p->n_range;
    a.f0 = p->freq_hz;
    a.c0 = p->c0;
    a.g = p->c_grad;
    a.alpha_db = p->abs_db_per_m;
    a.k_d = p->k_d;
    a.k_s = p->k_s;
    a.phong_n = p->phong_n;
    a.c_ref = p->c0 + p->c_grad * q->position[2];
    a.c_hi = p->c0 + fabs(p->c_grad) * (fmax((double)sc->s.zabs_max, fabs(q->position[2])) + 1.0);
    a.tan_h = p->hfov < M_PI ? tan(0.5 * p->hfov) : 0.0;
    a.tan_v = tan(0.5 * p->vfov);
    a.seed = p->seed;
    a.ping = q->ping;
    a.beams_h = beams_h_of(p);
    a.beams_v = beams_v_of(p);
    a.n_beams = a.beams_h * a.beams_v;
    a.n_r = p->rays_per_beam;
    a.log2_nr = ilog2(p->rays_per_beam);
    a.ne = 1 << (a.log2_nr / 2);
    a.na = a.n_r / a.ne;
    a.grid_mode = p->grid_mode;
    a.jitter = p->jitter;
    a.flags = p->flags;
    a.n_bins = p->n_range;
    a.K = p->max_bounces;
    a.n_rays = (int64_t)a.n_beams * a.n_r;
    a.volume = reinterpret_cast<float2 *>(volume);
    a.gbuf = gbuffer;
    a.incoh = incoh;
    if (rec) {
        a.rec_tri = rec->tri;
        a.rec_bin = rec->bin;
        a.rec_vis = rec->vis;
        a.rec_amp = reinterpret_cast<float2 *>(rec->amp);
        a.stats = rec->stats;
        a.rec_beam = rec->beam;
        a.rec_rbin = rec->retro_bin;
        a.rec_ramp = reinterpret_cast<float2 *>(rec->retro_amp);
    }
    a.mask = ray_mask;
    // a traversal of a valid hierarchy visits every node and every leaf at most once
    a.max_steps = (uint32_t)(sc->s.n_nodes + sc->s.n_tri + 64);
    return SONAR_OK;
}

sonar_status fill_detect_args(const sonar_cf32 *volume, const sonar_params *p, const sonar_pose *q,
                              const sonar_cfar *c, sonar_point *points, int32_t capacity, int32_t *dev_count,
                              void *workspace, size_t ws_bytes, sonar::DetectArgs *out)
{
    sonar_status st = check_params(p);
    if (st != SONAR_OK) return st;
    if ((st = check_pose(q)) != SONAR_OK) return st;
    if (!volume || !dev_count || !workspace) return fail(SONAR_E_INVALID, "volume, dev_count and workspace are required");
    if (!c) return fail(SONAR_E_INVALID, "cfar is NULL");
    if (c->train < 1 || c->guard < 0 || c->train > 64 || c->guard > 64)
        return fail(SONAR_E_INVALID, "train must be in [1, 64] and guard in [0, 64]");
    if (c->max_per_beam < 1 || c->max_per_beam > 16) return fail(SONAR_E_INVALID, "max_per_beam must be in [1, 16]");
    if (!(c->pfa > 0 && c->pfa < 1)) return fail(SONAR_E_INVALID, "pfa must be in (0, 1)");
    if (!(c->noise_floor >= 0) || !isfinite(c->noise_floor)) return fail(SONAR_E_INVALID, "noise_floor must be >= 0");
    if (capacity < 0 || (capacity > 0 && !points)) return fail(SONAR_E_INVALID, "points required when capacity > 0");
    int nb = beams_h_of(p) * beams_v_of(p);
    if (ws_bytes < sonar::detect_workspace_bytes(nb, 16))
        return fail(SONAR_E_INVALID, "workspace smaller than sonar_detect_workspace_size()");
    sonar::DetectArgs &a = *out;
    memset(&a, 0, sizeof(a));
    a.volume = reinterpret_cast<const float2 *>(volume);
    a.points = points;
    a.count = dev_count;
    char *w = (char *)workspace;
    size_t nb4 = ((size_t)nb + 3) & ~(size_t)3;
    a.beam_count = (int32_t *)w;
    a.beam_bins = (int32_t *)(w + sizeof(int32_t) * nb4);
    a.beam_pw = (float *)(w + sizeof(int32_t) * nb4 + sizeof(int32_t) * (size_t)nb * 16);
    // alpha(N) = N (pfa^(-1/N) - 1): the CA-CFAR scale for N exponential training cells
    a.alpha[0] = 0.0;
    for (int n = 1; n <= 2 * 64; ++n) a.alpha[n] = n * (pow(c->pfa, -1.0 / n) - 1.0);
    a.n_beams = nb;
    a.n_bins = p->n_range;
    a.beams_h = beams_h_of(p);
    a.grid_mode = p->grid_mode;
    a.train = c->train;
    a.guard = c->guard;
    a.max_per_beam = c->max_per_beam;
    a.capacity = capacity;
    a.pfa = c->pfa;
    a.noise_floor = c->noise_floor;
    a.hfov = p->hfov;
    a.vfov = p->vfov;
    a.dth_h = p->hfov / p->n_h;
    a.dth_v = p->vfov / p->n_v;
    a.r_min = p->r_min;
    a.dr = (p->r_max - p->r_min) / p->n_range;
    for (int i = 0; i < 3; ++i) a.pos[i] = q->position[i];
    for (int i = 0; i < 9; ++i) a.rot[i] = q->rot[i];
    return SONAR_OK;
}

}  // namespace

// Device scratch of sonar_ping_detect_noalloc: the detection workspace (and a
// receive-binning list) of one call, held by every GPU the library runs on
// until the process ends. Host code never uses the array's name as an
// address: each device's copy is resolved once through hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[SONAR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_SCRATCH_DEVICES] = {};

// The address of the current device's scratch (resolved on its first use).
sonar_status device_scratch(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_SCRATCH_DEVICES) return fail(SONAR_E_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SONAR_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SONAR_OK;
}

}  // namespace

extern "C" {

const char *sonar_last_error(void) { return g_err; }

const char *sonar_status_string(sonar_status s)
{
    switch (s) {
        case SONAR_OK: return "ok";
        case SONAR_W_TRUNCATED: return "output truncated to capacity";
        case SONAR_E_INVALID: return "invalid argument";
        case SONAR_E_NOMEM: return "out of device memory";
        case SONAR_E_DEVICE: return "device error";
        case SONAR_E_STACK: return "traversal stack overflow";
        case SONAR_E_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

sonar_status sonar_params_from_resolution(double hfov, double vfov, double dth_h, double dth_v, double r_min,
                                          double r_max, double dr, sonar_params *p)
{
    if (!p) return fail(SONAR_E_INVALID, "params is NULL");
    if (!(hfov > 0) || !(vfov > 0) || !(dth_h > 0) || !(dth_v > 0) || !(dr > 0) || !(r_max > r_min) ||
        !(r_min >= 0))
        return fail(SONAR_E_INVALID, "resolutions and fields of view must be positive, r_max > r_min >= 0");
    double nr = floor((r_max - r_min) / dr + 1e-9);
    double nh = floor(hfov / dth_h + 1e-9);
    double nv = floor(vfov / dth_v + 1e-9);
    if (nr < 1 || nh < 1 || nv < 1 || nr > sonar::MAX_BINS || nh > 65536 || nv > 65536)
        return fail(SONAR_E_INVALID, "resulting grid out of range");
    p->hfov = hfov;
    p->vfov = vfov;
    p->r_min = r_min;
    p->r_max = r_max;
    p->n_range = (int32_t)nr;
    p->n_h = (int32_t)nh;
    p->n_v = (int32_t)nv;
    return SONAR_OK;
}

sonar_status sonar_build_scene(const sonar_mesh *m, sonar_stream stream, sonar_scene **out)
{
    g_err[0] = 0;
    if (!out) return fail(SONAR_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!m) return fail(SONAR_E_INVALID, "mesh is NULL");
    if (!m->vertices || !m->indices || !m->reflectivity || !m->phase || !m->material)
        return fail(SONAR_E_INVALID, "mesh arrays must not be NULL");
    if (m->n_triangles < 1 || m->n_vertices < 3) return fail(SONAR_E_INVALID, "need >= 1 triangle, >= 3 vertices");
    if (m->n_triangles >= (int64_t)1 << 28) return fail(SONAR_E_INVALID, "at most 2^28 - 1 triangles");
    if (m->leaf_size < 0 || m->leaf_size > 8) return fail(SONAR_E_INVALID, "leaf_size must be in [0, 8]");
    sonar_mesh mm = *m;
    if (mm.leaf_size == 0) mm.leaf_size = 3;
    sonar_scene *sc = new (std::nothrow) sonar_scene();
    if (!sc) return fail(SONAR_E_NOMEM, "host allocation failed");
    if (hipGetDevice(&sc->s.device) != hipSuccess) {
        delete sc;
        return fail(SONAR_E_DEVICE, "no HIP device");
    }
    char err[256] = "";
    sonar_status st = sonar::build_hierarchy(mm, (hipStream_t)stream, &sc->s, err, sizeof(err));
    if (st != SONAR_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        free_scene_mem(sc->s);
        delete sc;
        return fail(st, "%s", err);
    }
    *out = sc;
    return SONAR_OK;
}

void sonar_free_scene(sonar_scene *sc)
{
    if (!sc) return;
    free_scene_mem(sc->s);
    delete sc;
}

sonar_status sonar_get_scene_info(const sonar_scene *sc, sonar_scene_info *info)
{
    if (!sc || !info) return fail(SONAR_E_INVALID, "scene or info is NULL");
    info->n_triangles = sc->s.n_tri;
    info->n_nodes = sc->s.n_nodes;
    info->depth = sc->s.depth;
    info->leaf_size = sc->s.leaf_size;
    for (int k = 0; k < 3; ++k) {
        info->lo[k] = sc->s.lo[k];
        info->hi[k] = sc->s.hi[k];
    }
    info->node_bytes = sc->s.n_nodes * 128;
    info->tri_bytes = sc->s.n_tri * 48;
    return SONAR_OK;
}

sonar_status sonar_ping(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q, sonar_cf32 *volume,
                        float *gbuffer, float *incoh, const sonar_ray_record *rec, const uint32_t *ray_mask,
                        sonar_stream stream)
{
    g_err[0] = 0;
    sonar::PingArgs a;
    sonar_status st = fill_ping_args(sc, p, q, volume, gbuffer, incoh, rec, ray_mask, &a);
    if (st != SONAR_OK) return st;
    if (needs_rx_list(p))
        return fail(SONAR_E_INVALID, "receive binning with several bounces needs a workspace: use sonar_ping_rx");
    hipError_t e = sonar::launch_ping(a, sc->s.stack, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "ping launch: %s", hipGetErrorString(e));
    return SONAR_OK;
}

static_assert(SONAR_MAX_SSP_KNOTS == sonar::MAX_SSP_KNOTS, "profile knots");

// Ping arguments through a layered profile: validation of the knots, the
// layers' gradients and offsets, the time-to-range speed at the sensor and
// an upper bound of c over the scene.
static sonar_status layered_args(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q,
                                 const sonar_ssp *ssp, sonar_cf32 *volume, float *gbuffer, float *incoh,
                                 const sonar_ray_record *rec, const uint32_t *ray_mask, sonar::PingArgs *out)
{
    if (!ssp) return fail(SONAR_E_INVALID, "ssp is NULL");
    if (!sc) return fail(SONAR_E_INVALID, "scene is NULL");
    sonar_status st = check_params(p);
    if (st != SONAR_OK) return st;
    if ((st = check_pose(q)) != SONAR_OK) return st;
    const int n = ssp->n_knots;
    if (n < 2 || n > SONAR_MAX_SSP_KNOTS)
        return fail(SONAR_E_INVALID, "n_knots must be in [2, %d]", SONAR_MAX_SSP_KNOTS);
    for (int k = 0; k < n; ++k) {
        if (!isfinite(ssp->z[k]) || !(ssp->c[k] > 0) || !isfinite(ssp->c[k]))
            return fail(SONAR_E_INVALID, "knot %d: z finite and c > 0 required", k);
        if (k > 0 && !(ssp->z[k] > ssp->z[k - 1])) return fail(SONAR_E_INVALID, "knot depths must increase");
    }
    const int nl = n - 1;
    double g[SONAR_MAX_SSP_KNOTS], c0[SONAR_MAX_SSP_KNOTS];
    for (int i = 0; i < nl; ++i) {
        g[i] = (ssp->c[i + 1] - ssp->c[i]) / (ssp->z[i + 1] - ssp->z[i]);
        c0[i] = ssp->c[i] - g[i] * ssp->z[i];
    }
    auto layer_of = [&](double z) {
        int i = 0;
        while (i + 1 < nl && z >= ssp->z[i + 1]) ++i;
        return i;
    };
    auto c_at = [&](double z) { const int i = layer_of(z); return c0[i] + g[i] * z; };
    // c over the scene and the sensor (1 m margin): its extremes are at the ends or at knots
    const double zmax = fmax((double)sc->s.zabs_max, fabs(q->position[2])) + 1.0;
    double c_lo = fmin(c_at(-zmax), c_at(zmax)), c_hi = fmax(c_at(-zmax), c_at(zmax));
    for (int k = 0; k < n; ++k)
        if (fabs(ssp->z[k]) <= zmax) {
            c_lo = fmin(c_lo, ssp->c[k]);
            c_hi = fmax(c_hi, ssp->c[k]);
        }
    if (!(c_lo > 0.0)) return fail(SONAR_E_INVALID, "the profile's sound speed must stay positive over the scene");
    for (int i = 0; i < nl; ++i)
        if (fabs(g[i]) * 2.0 * p->r_max / c_lo > 1e-2)
            return fail(SONAR_E_UNSUPPORTED, "layer %d bends too strongly for one chord per layer", i);
    sonar_params pp = *p;
    pp.c_grad = 0.0;
    pp.c0 = c_at(q->position[2]);
    sonar::PingArgs &a = *out;
    st = fill_ping_args(sc, &pp, q, volume, gbuffer, incoh, rec, ray_mask, &a);
    if (st != SONAR_OK) return st;
    a.n_layers = nl;
    for (int k = 0; k < n; ++k) a.lay_z[k] = ssp->z[k];
    for (int i = 0; i < nl; ++i) {
        a.lay_g[i] = g[i];
        a.lay_c0[i] = c0[i];
    }
    a.c_ref = pp.c0;
    a.c_hi = c_hi;
    return SONAR_OK;
}

// A ping through a layered profile; `workspace` (NULL: none) holds the
// receive-binning list of several bounces.
static sonar_status ping_ssp(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q, const sonar_ssp *ssp,
                             sonar_cf32 *volume, float *gbuffer, float *incoh, const sonar_ray_record *rec,
                             const uint32_t *ray_mask, void *workspace, size_t ws_bytes, sonar_stream stream)
{
    sonar::PingArgs a;
    sonar_status st = layered_args(sc, p, q, ssp, volume, gbuffer, incoh, rec, ray_mask, &a);
    if (st != SONAR_OK) return st;
    if (needs_rx_list(p)) {
        if (!workspace)
            return fail(SONAR_E_INVALID, "receive binning with several bounces needs a workspace: use sonar_ping_ssp_rx");
        if (ws_bytes < rx_bytes(p)) return fail(SONAR_E_INVALID, "workspace smaller than sonar_rx_workspace_size()");
        if (((uintptr_t)workspace & 255) != 0) return fail(SONAR_E_INVALID, "workspace must be 256-byte aligned");
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (needs_rx_list(p)) {
        // reset -> ping -> scatter of the returns binned to other beams
        set_rx_area(a, p, workspace);
        e = sonar::launch_rx_reset(a.rx_count, s);
    }
    if (e == hipSuccess) e = sonar::launch_ping_layered(a, sc->s.stack, s);
    if (e == hipSuccess && a.rx_list) e = sonar::launch_rx_scatter(a, s);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "ping launch: %s", hipGetErrorString(e));
    return SONAR_OK;
}

sonar_status sonar_ping_ssp(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q, const sonar_ssp *ssp,
                            sonar_cf32 *volume, float *gbuffer, float *incoh, const sonar_ray_record *rec,
                            const uint32_t *ray_mask, sonar_stream stream)
{
    g_err[0] = 0;
    return ping_ssp(sc, p, q, ssp, volume, gbuffer, incoh, rec, ray_mask, nullptr, 0, stream);
}

sonar_status sonar_ping_ssp_rx(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q, const sonar_ssp *ssp,
                               sonar_cf32 *volume, float *gbuffer, float *incoh, const sonar_ray_record *rec,
                               const uint32_t *ray_mask, void *workspace, size_t ws_bytes, sonar_stream stream)
{
    g_err[0] = 0;
    return ping_ssp(sc, p, q, ssp, volume, gbuffer, incoh, rec, ray_mask, workspace, ws_bytes, stream);
}

size_t sonar_rx_workspace_size(const sonar_params *p)
{
    if (check_params(p) != SONAR_OK) return 0;
    return needs_rx_list(p) ? rx_bytes(p) : 256;
}

sonar_status sonar_ping_rx(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q, sonar_cf32 *volume,
                           float *gbuffer, float *incoh, const sonar_ray_record *rec, const uint32_t *ray_mask,
                           void *workspace, size_t ws_bytes, sonar_stream stream)
{
    g_err[0] = 0;
    sonar::PingArgs a;
    sonar_status st = fill_ping_args(sc, p, q, volume, gbuffer, incoh, rec, ray_mask, &a);
    if (st != SONAR_OK) return st;
    if (needs_rx_list(p)) {
        if (!workspace || ws_bytes < rx_bytes(p))
            return fail(SONAR_E_INVALID, "workspace smaller than sonar_rx_workspace_size()");
        if (((uintptr_t)workspace & 255) != 0) return fail(SONAR_E_INVALID, "workspace must be 256-byte aligned");
        set_rx_area(a, p, workspace);
    }
    hipError_t e = launch_ping_rx(a, sc->s.stack, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "ping launch: %s", hipGetErrorString(e));
    return SONAR_OK;
}

size_t sonar_workspace_size(const sonar_scene *sc, const sonar_params *p, int32_t n_pings)
{
    if (!sc || n_pings < 1 || check_params(p) != SONAR_OK) return 0;
    const size_t one = (needs_rx_list(p) ? ((rx_bytes(p) + 255) & ~(size_t)255) : 0) + staged_bytes(p);
    return one * (size_t)n_pings;
}

sonar_status sonar_ping_ws(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q, sonar_cf32 *volume,
                           float *gbuffer, float *incoh, const sonar_ray_record *rec, const uint32_t *ray_mask,
                           void *workspace, size_t ws_bytes, sonar_stream stream)
{
    g_err[0] = 0;
    sonar::PingArgs a;
    sonar_status st = fill_ping_args(sc, p, q, volume, gbuffer, incoh, rec, ray_mask, &a);
    if (st != SONAR_OK) return st;
    const size_t need = sonar_workspace_size(sc, p, 1);
    if (need > 0 && (!workspace || ws_bytes < need))
        return fail(SONAR_E_INVALID, "workspace smaller than sonar_workspace_size()");
    if (need > 0 && ((uintptr_t)workspace & 255) != 0) return fail(SONAR_E_INVALID, "workspace must be 256-byte aligned");
    char *w = reinterpret_cast<char *>(workspace);
    if (needs_rx_list(p)) {
        set_rx_area(a, p, w);
        w += (rx_bytes(p) + 255) & ~(size_t)255;
    }
    // the counting kernels are fused ones: with counters the staged area stays unused
    if (staged_bytes(p) > 0 && !a.stats) sonar::set_staged_area(a, w);
    hipError_t e = launch_ping_rx(a, sc->s.stack, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "ping launch: %s", hipGetErrorString(e));
    return SONAR_OK;
}

// detection workspace, then (receive binning with several bounces) the list area
static size_t det_bytes(const sonar_params *p)
{
    return (sonar::detect_workspace_bytes(beams_h_of(p) * beams_v_of(p), 16) + 255) & ~(size_t)255;
}

// rx list area rounded so that a staged area after it stays aligned
static size_t rx_bytes_aligned(const sonar_params *p)
{
    return needs_rx_list(p) ? (rx_bytes(p) + 255) & ~(size_t)255 : 0;
}

size_t sonar_detect_workspace_size(const sonar_params *p)
{
    if (check_params(p) != SONAR_OK) return 0;
    return det_bytes(p) + rx_bytes_aligned(p) + staged_bytes(p);
}

sonar_status sonar_detect(const sonar_cf32 *volume, const sonar_params *p, const sonar_pose *q,
                          const sonar_cfar *c, sonar_point *points, int32_t capacity, int32_t *dev_count,
                          void *workspace, size_t ws_bytes, sonar_stream stream)
{
    g_err[0] = 0;
    sonar::DetectArgs a;
    sonar_status st = fill_detect_args(volume, p, q, c, points, capacity, dev_count, workspace, ws_bytes, &a);
    if (st != SONAR_OK) return st;
    hipError_t e = sonar::launch_detect(a, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "detect launch: %s", hipGetErrorString(e));
    return SONAR_OK;
}

// Ping + detection into a given workspace (the caller's, or the static
// scratch of the allocation-free entry point).
static sonar_status ping_detect_into(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q,
                                     const sonar_cfar *c, sonar_cf32 *volume, sonar_point *points, int32_t capacity,
                                     int32_t *dev_count, void *workspace, size_t ws_bytes, hipStream_t s)
{
    sonar::PingArgs pa;
    sonar_status st = fill_ping_args(sc, p, q, volume, nullptr, nullptr, nullptr, nullptr, &pa);
    if (st != SONAR_OK) return st;
    sonar::DetectArgs da;
    st = fill_detect_args(volume, p, q, c, points, capacity, dev_count, workspace, ws_bytes, &da);
    if (st != SONAR_OK) return st;
    // several bounces with a workspace that holds the staged area: the staged kernels
    const size_t stg = staged_bytes(p);
    if (stg > 0 && ws_bytes >= det_bytes(p) + rx_bytes_aligned(p) + stg && ((uintptr_t)workspace & 255) == 0)
        sonar::set_staged_area(pa, reinterpret_cast<char *>(workspace) + det_bytes(p) + rx_bytes_aligned(p));
    if (needs_rx_list(p)) {
        // moved returns land after the ping kernel: detection runs after them
        if (ws_bytes < det_bytes(p) + rx_bytes(p) || ((uintptr_t)workspace & 255) != 0)
            return fail(SONAR_E_INVALID, "workspace smaller than sonar_detect_workspace_size() or not 256-byte aligned");
        set_rx_area(pa, p, reinterpret_cast<char *>(workspace) + det_bytes(p));
        hipError_t e = launch_ping_rx(pa, sc->s.stack, s);
        if (e == hipSuccess) e = sonar::launch_detect(da, s);
        if (e != hipSuccess) return fail(SONAR_E_DEVICE, "ping/detect launch: %s", hipGetErrorString(e));
        return SONAR_OK;
    }
    // the fused test needs alpha(N) > 1 for every window size, so that a bin
    // without a return can never be detected
    bool fused = true;
    for (int n = 1; n <= 2 * c->train; ++n)
        if (!(da.alpha[n] > 1.0)) fused = false;
    hipError_t e;
    if (fused) {
        pa.det_count = da.beam_count;
        pa.det_bins = da.beam_bins;
        pa.det_pw = da.beam_pw;
        pa.det_G = c->guard;
        pa.det_T = c->train;
        pa.det_M = c->max_per_beam;
        pa.det_n0 = (float)c->noise_floor;
        for (int n = 0; n <= 2 * 64; ++n) pa.det_alpha[n] = da.alpha[n];
        e = launch_any(pa, sc->s.stack, s);
        if (e == hipSuccess) e = sonar::launch_emit(da, s);
    } else {
        e = launch_any(pa, sc->s.stack, s);
        if (e == hipSuccess) e = sonar::launch_detect(da, s);
    }
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "ping/detect launch: %s", hipGetErrorString(e));
    return SONAR_OK;
}

sonar_status sonar_ping_detect(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q,
                               const sonar_cfar *c, sonar_cf32 *volume, sonar_point *points, int32_t capacity,
                               int32_t *dev_count, void *workspace, size_t ws_bytes, sonar_stream stream)
{
    g_err[0] = 0;
    return ping_detect_into(sc, p, q, c, volume, points, capacity, dev_count, workspace, ws_bytes,
                            (hipStream_t)stream);
}

sonar_status sonar_ping_detect_noalloc(const sonar_scene *sc, const sonar_params *p, const sonar_pose *q,
                                       const sonar_cfar *c, sonar_cf32 *volume, sonar_point *points,
                                       int32_t capacity, int32_t *dev_count, sonar_stream stream)
{
    g_err[0] = 0;
    if (!sc) return fail(SONAR_E_INVALID, "scene is NULL");
    sonar_status st = check_params(p);
    if (st != SONAR_OK) return st;
    const size_t need = det_bytes(p) + (needs_rx_list(p) ? rx_bytes(p) : 0);
    if (need > SONAR_NOALLOC_SCRATCH_BYTES)
        return fail(SONAR_E_INVALID, "these parameters need %zu bytes of scratch, more than the %zu of "
                                     "sonar_ping_detect_noalloc (use sonar_ping_detect with a workspace)",
                    need, (size_t)SONAR_NOALLOC_SCRATCH_BYTES);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev != sc->s.device) return fail(SONAR_E_INVALID, "the scene's device (%d) must be current, not %d",
                                         sc->s.device, dev);
    void *ws = nullptr;
    if ((st = device_scratch(&ws)) != SONAR_OK) return st;
    return ping_detect_into(sc, p, q, c, volume, points, capacity, dev_count, ws, SONAR_NOALLOC_SCRATCH_BYTES,
                            (hipStream_t)stream);
}

sonar_status sonar_add_reverb(sonar_cf32 *volume, const sonar_params *p, const sonar_pose *q,
                              const sonar_reverb *rv, sonar_stream stream)
{
    g_err[0] = 0;
    sonar_status st = check_params(p);
    if (st != SONAR_OK) return st;
    if ((st = check_pose(q)) != SONAR_OK) return st;
    if (!volume || !rv) return fail(SONAR_E_INVALID, "volume and reverb are required");
    if (p->grid_mode != 0) return fail(SONAR_E_UNSUPPORTED, "reverberation needs cell-centred beams (grid_mode 0)");
    if (!isfinite(rv->sv_db) || !(rv->noise_power >= 0) || !isfinite(rv->noise_power))
        return fail(SONAR_E_INVALID, "sv_db must be finite and noise_power finite and >= 0");
    sonar::ReverbArgs a;
    a.volume = reinterpret_cast<float2 *>(volume);
    a.beams_h = beams_h_of(p);
    a.n_beams = (int64_t)a.beams_h * beams_v_of(p);
    a.n_bins = p->n_range;
    a.r_min = (float)p->r_min;
    a.dr = (float)((p->r_max - p->r_min) / p->n_range);
    a.vfov = (float)p->vfov;
    a.dth_v = (float)(p->vfov / p->n_v);
    a.cell_solid = (float)((p->hfov / p->n_h) * (p->vfov / p->n_v));
    a.sv = (float)pow(10.0, rv->sv_db / 10.0);
    a.alpha_db = (float)p->abs_db_per_m;
    a.noise = (float)rv->noise_power;
    a.seed = rv->seed;
    a.ping = q->ping;
    hipError_t e = sonar::launch_reverb(a, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "reverberation launch: %s", hipGetErrorString(e));
    return SONAR_OK;
}

static_assert(SONAR_MAX_PULSE_TAPS == sonar::MAX_PULSE_TAPS, "pulse tap bound");
static_assert(SONAR_MAX_PULSE_BINS == sonar::MAX_PULSE_BINS, "pulse bin bound");

sonar_status sonar_pulse_dt(const sonar_params *p, const sonar_pose *q, const sonar_ssp *ssp, double *dt)
{
    g_err[0] = 0;
    if (!dt) return fail(SONAR_E_INVALID, "dt is NULL");
    sonar_status st = check_params(p);
    if (st != SONAR_OK) return st;
    if ((st = check_pose(q)) != SONAR_OK) return st;
    const double z = q->position[2];
    double c;
    if (ssp) {
        // the layer holding the sensor depth (a point on a knot belongs to the layer above)
        const int n = ssp->n_knots;
        if (n < 2 || n > SONAR_MAX_SSP_KNOTS)
            return fail(SONAR_E_INVALID, "n_knots must be in [2, %d]", SONAR_MAX_SSP_KNOTS);
        for (int k = 0; k < n; ++k) {
            if (!isfinite(ssp->z[k]) || !(ssp->c[k] > 0) || !isfinite(ssp->c[k]))
                return fail(SONAR_E_INVALID, "knot %d: z finite and c > 0 required", k);
            if (k > 0 && !(ssp->z[k] > ssp->z[k - 1])) return fail(SONAR_E_INVALID, "knot depths must increase");
        }
        int i = 0;
        while (i + 1 < n - 1 && z >= ssp->z[i + 1]) ++i;
        const double g = (ssp->c[i + 1] - ssp->c[i]) / (ssp->z[i + 1] - ssp->z[i]);
        c = ssp->c[i] + g * (z - ssp->z[i]);
    } else {
        c = p->c0 + p->c_grad * z;
    }
    if (!(c > 0.0) || !isfinite(c)) return fail(SONAR_E_INVALID, "sound speed at the sensor must be positive");
    *dt = 2.0 * ((p->r_max - p->r_min) / p->n_range) / c;
    return SONAR_OK;
}

sonar_status sonar_lfm_pulse(double bandwidth_hz, double duration_s, double dt_s, int32_t window, sonar_cf32 *taps,
                             int32_t max_len, int32_t *len)
{
    g_err[0] = 0;
    if (!taps || !len) return fail(SONAR_E_INVALID, "taps and len are required");
    if (!(bandwidth_hz >= 0.0) || !(duration_s > 0.0) || !(dt_s > 0.0) || (window != 0 && window != 1))
        return fail(SONAR_E_INVALID, "need bandwidth >= 0, duration > 0, dt > 0, window 0 or 1");
    const double q = duration_s / dt_s;
    if (!(q < 1e9)) return fail(SONAR_E_INVALID, "duration / dt too large");
    int L = (int)llround(q);
    if (L < 1) L = 1;
    if (L > SONAR_MAX_PULSE_TAPS || L > max_len)
        return fail(SONAR_E_INVALID, "pulse of %d taps: at most %d (and max_len %d)", L, SONAR_MAX_PULSE_TAPS, max_len);
    const double rate = bandwidth_hz / duration_s, pi = 3.14159265358979323846;
    for (int k = 0; k < L; ++k) {
        const double t = (k + 0.5) * dt_s - 0.5 * L * dt_s;
        const double sw = sin(pi * (k + 0.5) / L);
        const double w = window == 0 ? 1.0 : sw * sw;
        const double ph = pi * rate * t * t;
        taps[k].re = (float)(w * cos(ph));
        taps[k].im = (float)(w * sin(ph));
    }
    *len = L;
    return SONAR_OK;
}

static bool ranges_overlap(const void *a, const void *b, size_t bytes)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bytes && y < x + bytes;
}

sonar_status sonar_pulse_compress(const sonar_cf32 *volume, int64_t n_beams, int32_t n_bins, const sonar_cf32 *pulse,
                                  int32_t pulse_len, sonar_cf32 *series, sonar_cf32 *matched, sonar_stream stream)
{
    g_err[0] = 0;
    if (!volume || !pulse) return fail(SONAR_E_INVALID, "volume and pulse are required");
    if (!series && !matched) return fail(SONAR_E_INVALID, "at least one of series and matched is required");
    if (n_beams < 0 || n_beams >= ((int64_t)1 << 31)) return fail(SONAR_E_INVALID, "n_beams must be in [0, 2^31)");
    if (n_bins < 1 || n_bins > SONAR_MAX_PULSE_BINS)
        return fail(SONAR_E_INVALID, "n_bins must be in [1, %d]", SONAR_MAX_PULSE_BINS);
    if (pulse_len < 1 || pulse_len > SONAR_MAX_PULSE_TAPS)
        return fail(SONAR_E_INVALID, "pulse_len must be in [1, %d]", SONAR_MAX_PULSE_TAPS);
    const size_t bytes = (size_t)n_beams * (size_t)n_bins * sizeof(sonar_cf32);
    if ((series && ranges_overlap(series, volume, bytes)) || (matched && ranges_overlap(matched, volume, bytes)) ||
        (series && matched && ranges_overlap(series, matched, bytes)))
        return fail(SONAR_E_INVALID, "outputs overlap the input or each other");
    sonar::PulseArgs a;
    a.x = reinterpret_cast<const float2 *>(volume);
    a.s = reinterpret_cast<float2 *>(series);
    a.y = reinterpret_cast<float2 *>(matched);
    a.n_beams = n_beams;
    a.n_bins = n_bins;
    a.L = pulse_len;
    for (int k = 0; k < sonar::MAX_PULSE_TAPS; ++k)
        a.p[k] = k < pulse_len ? make_float2(pulse[k].re, pulse[k].im) : make_float2(0.f, 0.f);
    hipError_t e = sonar::launch_pulse(a, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "pulse compression launch: %s", hipGetErrorString(e));
    return SONAR_OK;
}

size_t sonar_batch_desc_bytes(void) { return sizeof(sonar::PingArgs); }

size_t sonar_batch_emit_desc_bytes(void) { return sizeof(sonar::DetectArgs); }

// Detection workspace of one ping, rounded so that every slice stays aligned.
static size_t det_slice_bytes(const sonar_params *p)
{
    size_t b = sonar_detect_workspace_size(p);
    return (b + 255) & ~(size_t)255;
}

size_t sonar_batch_detect_workspace_size(int32_t n, const sonar_params *params)
{
    if (n < 1 || !params) return 0;
    size_t total = 0;
    for (int32_t i = 0; i < n; ++i) {
        const size_t b = det_slice_bytes(&params[i]);
        if (b == 0) return 0;
        total += b;
    }
    return total;
}

sonar_status sonar_batch_prepare_detect(int32_t n, const sonar_params *params, const sonar_pose *poses,
                                       const sonar_cfar *cfar, sonar_point *const *points, const int32_t *capacity,
                                       int32_t *dev_counts, void *workspace, size_t ws_bytes, void *host_desc,
                                       void *host_emit)
{
    g_err[0] = 0;
    if (n < 1 || !params || !poses || !cfar || !points || !capacity || !dev_counts || !workspace || !host_desc ||
        !host_emit)
        return fail(SONAR_E_INVALID, "all arguments are required (n_pings >= 1)");
    const size_t need = sonar_batch_detect_workspace_size(n, params);
    if (need == 0 || ws_bytes < need) return fail(SONAR_E_INVALID, "workspace smaller than sonar_batch_detect_workspace_size()");
    sonar::PingArgs *d = reinterpret_cast<sonar::PingArgs *>(host_desc);
    sonar::DetectArgs *em = reinterpret_cast<sonar::DetectArgs *>(host_emit);
    char *w = reinterpret_cast<char *>(workspace);
    for (int32_t i = 0; i < n; ++i) {
        const size_t slice = det_slice_bytes(&params[i]);
        sonar::DetectArgs da;
        sonar_status st = fill_detect_args(reinterpret_cast<const sonar_cf32 *>(d[i].volume), &params[i], &poses[i],
                                           cfar, points[i], capacity[i], dev_counts + i, w, slice, &da);
        if (st != SONAR_OK) {
            char tmp[512];
            snprintf(tmp, sizeof(tmp), "ping %d: %s", i, g_err);
            return fail(st, "%s", tmp);
        }
        if (da.n_beams != d[i].n_beams || da.n_bins != d[i].n_bins)
            return fail(SONAR_E_INVALID, "ping %d: parameters differ from the prepared batch", i);
        if (d[i].rx_list)
            return fail(SONAR_E_UNSUPPORTED, "ping %d: receive binning with several bounces moves returns after the "
                                             "in-kernel test: use sonar_detect per ping", i);
        for (int k = 1; k <= 2 * cfar->train; ++k)
            if (!(da.alpha[k] > 1.0))
                return fail(SONAR_E_UNSUPPORTED, "alpha(N) <= 1 for N = %d: use sonar_detect per ping", k);
        d[i].det_count = da.beam_count;
        d[i].det_bins = da.beam_bins;
        d[i].det_pw = da.beam_pw;
        d[i].det_G = cfar->guard;
        d[i].det_T = cfar->train;
        d[i].det_M = cfar->max_per_beam;
        d[i].det_n0 = (float)cfar->noise_floor;
        for (int k = 0; k <= 2 * 64; ++k) d[i].det_alpha[k] = da.alpha[k];
        em[i] = da;
        w += slice;
    }
    return SONAR_OK;
}

size_t sonar_batch_workspace_size(int32_t n_pings)
{
    if (n_pings < 1) return 0;
    return 256 + 2 * sizeof(unsigned long long) * (size_t)n_pings;
}

// Bytes of a batch's receive-binning lists: each ping's area (as for one
// ping), 256-byte aligned, in ping order.
static size_t batch_rx_bytes(int32_t n, const sonar_params *params)
{
    size_t total = 0;
    for (int32_t i = 0; i < n; ++i)
        if (needs_rx_list(&params[i])) total += (rx_bytes(&params[i]) + 255) & ~(size_t)255;
    return total;
}

size_t sonar_batch_rx_workspace_size(int32_t n_pings, const sonar_params *params)
{
    if (n_pings < 1 || !params) return 0;
    for (int32_t i = 0; i < n_pings; ++i)
        if (check_params(&params[i]) != SONAR_OK) return 0;
    return batch_rx_bytes(n_pings, params);
}

// Descriptors of a batch; `ssp` (NULL: none) is the layered profile every
// ping goes through, `rx_ws` holds the receive-binning lists.
static sonar_status batch_prepare(const sonar_scene *sc, int32_t n, const sonar_params *params,
                                  const sonar_pose *poses, const sonar_ssp *ssp, sonar_cf32 *const *volumes,
                                  void *rx_ws, size_t rx_ws_bytes, void *host_desc, sonar_batch_plan *plan)
{
    if (!sc || !params || !poses || !volumes || !host_desc || !plan)
        return fail(SONAR_E_INVALID, "scene, params, poses, volumes, host_desc and plan are required");
    if (n < 1) return fail(SONAR_E_INVALID, "n_pings must be >= 1");
    sonar::PingArgs *d = reinterpret_cast<sonar::PingArgs *>(host_desc);
    int64_t tiles = 0, rays = 0;
    int max_bins = 0, max_beams = 0;
    if (rx_ws && ((uintptr_t)rx_ws & 255) != 0) return fail(SONAR_E_INVALID, "workspace must be 256-byte aligned");
    size_t rx_off = 0;
    for (int32_t i = 0; i < n; ++i) {
        if ((params[i].flags & SONAR_FLAG_RETRO_CHAIN) != (params[0].flags & SONAR_FLAG_RETRO_CHAIN))
            return fail(SONAR_E_INVALID, "ping %d: the pings of a batch all take retro-chain returns or none", i);
        sonar_status st = ssp ? layered_args(sc, &params[i], &poses[i], ssp, volumes[i], nullptr, nullptr, nullptr,
                                             nullptr, &d[i])
                              : fill_ping_args(sc, &params[i], &poses[i], volumes[i], nullptr, nullptr, nullptr,
                                               nullptr, &d[i]);
        if (st != SONAR_OK) {
            char tmp[512];
            snprintf(tmp, sizeof(tmp), "ping %d: %s", i, g_err);
            return fail(st, "%s", tmp);
        }
        if (params[i].max_bounces != params[0].max_bounces ||
            (!ssp && (params[i].c_grad != 0.0) != (params[0].c_grad != 0.0)))
            return fail(SONAR_E_INVALID, "ping %d: a batch needs one max_bounces and one medium type", i);
        if (needs_rx_list(&params[i])) {
            if (!rx_ws)
                return fail(SONAR_E_UNSUPPORTED, "ping %d: receive binning with several bounces needs the list "
                                                 "workspace of sonar_batch_prepare_rx", i);
            const size_t need = (rx_bytes(&params[i]) + 255) & ~(size_t)255;
            if (rx_off + need > rx_ws_bytes)
                return fail(SONAR_E_INVALID, "workspace smaller than sonar_batch_rx_workspace_size()");
            set_rx_area(d[i], &params[i], reinterpret_cast<char *>(rx_ws) + rx_off);
            rx_off += need;
        }
        int64_t t = (d[i].n_rays + 255) / 256;
        if (tiles + t > 0x7FFFFFFF) return fail(SONAR_E_INVALID, "batch too large");
        d[i].tile_offset = (int)tiles;
        d[i].n_tiles = (int)t;
        tiles += t;
        rays += d[i].n_rays;
        if (d[i].n_bins > max_bins) max_bins = d[i].n_bins;
        if (d[i].n_beams > max_beams) max_beams = (int)d[i].n_beams;
    }
    plan->n_pings = n;
    plan->max_bounces = params[0].max_bounces;
    plan->arc = ssp ? 2 : (params[0].c_grad != 0.0 ? 1 : 0);
    plan->max_bins = max_bins;
    plan->max_beams = max_beams;
    plan->retro = (params[0].flags & SONAR_FLAG_RETRO_CHAIN) && params[0].max_bounces > 1;
    int32_t n_rx = 0;
    for (int32_t i = 0; i < n; ++i) n_rx += d[i].rx_list != nullptr;
    plan->rx = n_rx;
    plan->total_tiles = tiles;
    plan->total_rays = rays;
    return SONAR_OK;
}

sonar_status sonar_batch_prepare(const sonar_scene *sc, int32_t n, const sonar_params *params,
                                 const sonar_pose *poses, sonar_cf32 *const *volumes, void *host_desc,
                                 sonar_batch_plan *plan)
{
    g_err[0] = 0;
    return batch_prepare(sc, n, params, poses, nullptr, volumes, nullptr, 0, host_desc, plan);
}

sonar_status sonar_batch_prepare_ssp(const sonar_scene *sc, int32_t n, const sonar_params *params,
                                     const sonar_pose *poses, const sonar_ssp *ssp, sonar_cf32 *const *volumes,
                                     void *host_desc, sonar_batch_plan *plan)
{
    g_err[0] = 0;
    if (!ssp) return fail(SONAR_E_INVALID, "ssp is NULL");
    return batch_prepare(sc, n, params, poses, ssp, volumes, nullptr, 0, host_desc, plan);
}

sonar_status sonar_batch_prepare_rx(const sonar_scene *sc, int32_t n, const sonar_params *params,
                                    const sonar_pose *poses, const sonar_ssp *ssp, sonar_cf32 *const *volumes,
                                    void *rx_workspace, size_t rx_ws_bytes, void *host_desc, sonar_batch_plan *plan)
{
    g_err[0] = 0;
    return batch_prepare(sc, n, params, poses, ssp, volumes, rx_workspace, rx_ws_bytes, host_desc, plan);
}

sonar_status sonar_batch_set_outputs(void *host_desc, int32_t n_pings, int32_t ping, float *gbuffer, float *incoh,
                                     const sonar_ray_record *record, const uint32_t *ray_mask)
{
    g_err[0] = 0;
    if (!host_desc || ping < 0 || ping >= n_pings) return fail(SONAR_E_INVALID, "host_desc and 0 <= ping < n_pings are required");
    if (record && (!record->tri || !record->bin || !record->vis || !record->amp))
        return fail(SONAR_E_INVALID, "record arrays tri, bin, vis and amp must all be set");
    if (record && record->stats)
        return fail(SONAR_E_UNSUPPORTED, "traversal counters are not kept in batches");
    if (record && (!record->retro_bin) != (!record->retro_amp))
        return fail(SONAR_E_INVALID, "record arrays retro_bin and retro_amp go together");
    sonar::PingArgs &a = reinterpret_cast<sonar::PingArgs *>(host_desc)[ping];
    if (a.n_beams < 1 || a.n_r < 1 || a.n_tiles < 1) return fail(SONAR_E_INVALID, "descriptor %d is not a prepared one", ping);
    a.gbuf = gbuffer;
    a.incoh = incoh;
    a.rec_tri = record ? record->tri : nullptr;
    a.rec_bin = record ? record->bin : nullptr;
    a.rec_vis = record ? record->vis : nullptr;
    a.rec_amp = record ? reinterpret_cast<float2 *>(record->amp) : nullptr;
    a.rec_beam = record ? record->beam : nullptr;
    a.rec_rbin = record ? record->retro_bin : nullptr;
    a.rec_ramp = record ? reinterpret_cast<float2 *>(record->retro_amp) : nullptr;
    a.stats = nullptr;
    a.mask = ray_mask;
    return SONAR_OK;
}

static sonar_status batch_launch_args(const sonar_scene *sc, const sonar_batch_plan *plan, const void *dev_desc,
                                      const sonar_batch_options *opt, void *ws, size_t ws_bytes,
                                      sonar::BatchLaunch *b)
{
    if (!sc || !plan || !dev_desc || !ws) return fail(SONAR_E_INVALID, "scene, plan, dev_desc and workspace are required");
    if (plan->n_pings < 1 || plan->max_bounces < 1 || plan->max_bounces > sonar::MAX_BOUNCES ||
        plan->max_bins < 1 || plan->max_bins > sonar::MAX_BINS || plan->total_tiles < 1)
        return fail(SONAR_E_INVALID, "plan is not one filled by sonar_batch_prepare");
    if (ws_bytes < sonar_batch_workspace_size(plan->n_pings)) return fail(SONAR_E_INVALID, "workspace too small");
    if (opt && (opt->blocks_per_cu < 0 || opt->blocks_per_cu > 64 || opt->tiles_per_item < 0 || opt->tiles_per_item > 64))
        return fail(SONAR_E_INVALID, "options out of range");
    if (opt && opt->waves_per_block != 0 && opt->waves_per_block != 1 && opt->waves_per_block != 2 &&
        opt->waves_per_block != 4)
        return fail(SONAR_E_INVALID, "waves_per_block must be 1, 2 or 4 (0: 4)");
    char *w = (char *)ws;
    b->desc = reinterpret_cast<const sonar::PingArgs *>(dev_desc);
    b->n_pings = plan->n_pings;
    if (plan->arc < 0 || plan->arc > 2) return fail(SONAR_E_INVALID, "plan is not one filled by sonar_batch_prepare");
    b->K = plan->max_bounces;
    b->arc = plan->arc != 0;
    b->layered = plan->arc == 2;
    b->retro = plan->retro != 0;
    b->rx = plan->rx != 0;
    b->depth = sc->s.stack;
    b->max_bins = plan->max_bins;
    b->total_tiles = plan->total_tiles;
    b->queue = reinterpret_cast<uint32_t *>(w);
    b->t0 = reinterpret_cast<unsigned long long *>(w + 256);
    b->t1 = b->t0 + plan->n_pings;
    b->blocks_per_cu = opt ? opt->blocks_per_cu : 0;
    b->tiles_per_item = opt && opt->tiles_per_item > 0 ? opt->tiles_per_item : 1;
    // layered and retro-chain batches have the 4-wave instantiations only
    b->waves_per_block = opt && opt->waves_per_block > 0 && !(plan->arc == 2 || plan->retro) ? opt->waves_per_block : 4;
    b->emit = opt ? reinterpret_cast<const sonar::DetectArgs *>(opt->emit_desc) : nullptr;
    b->max_beams = plan->max_beams;
    if (b->emit && plan->max_beams < 1) return fail(SONAR_E_INVALID, "plan has no beam count (prepare it again)");
    return SONAR_OK;
}

// The pings of a batch, then its batched point emission when it has one.
static hipError_t batch_launch_all(const sonar::BatchLaunch &b, hipStream_t s)
{
    hipError_t e = sonar::launch_ping_batch(b, s);
    if (e == hipSuccess && b.emit) e = sonar::launch_emit_batch(b.emit, b.n_pings, b.max_beams, s);
    return e;
}

sonar_status sonar_ping_batch(const sonar_scene *sc, const sonar_batch_plan *plan, const void *dev_desc,
                              const sonar_batch_options *opt, void *ws, size_t ws_bytes, sonar_stream stream)
{
    g_err[0] = 0;
    sonar::BatchLaunch b;
    sonar_status st = batch_launch_args(sc, plan, dev_desc, opt, ws, ws_bytes, &b);
    if (st != SONAR_OK) return st;
    hipError_t e = batch_launch_all(b, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "batch launch: %s", hipGetErrorString(e));
    return SONAR_OK;
}

sonar_status sonar_batch_stamps(const void *ws, int32_t n, uint64_t *start, uint64_t *finish, sonar_stream stream)
{
    if (!ws || n < 1 || !start || !finish) return fail(SONAR_E_INVALID, "workspace, n_pings and outputs are required");
    hipStream_t s = (hipStream_t)stream;
    const char *w = (const char *)ws;
    if (hipMemcpyAsync(start, w + 256, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(finish, w + 256 + sizeof(uint64_t) * n, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(SONAR_E_DEVICE, "stamp copy failed");
    return SONAR_OK;
}

sonar_status sonar_batch_graph_create(const sonar_scene *sc, const sonar_batch_plan *plan, const void *dev_desc,
                                      const sonar_batch_options *opt, void *ws, size_t ws_bytes, sonar_graph **out)
{
    g_err[0] = 0;
    if (!out) return fail(SONAR_E_INVALID, "out is NULL");
    *out = nullptr;
    sonar::BatchLaunch b;
    sonar_status st = batch_launch_args(sc, plan, dev_desc, opt, ws, ws_bytes, &b);
    if (st != SONAR_OK) return st;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return fail(SONAR_E_DEVICE, "capture stream creation failed");
    sonar_graph *g = new (std::nothrow) sonar_graph();
    if (!g) {
        (void)hipStreamDestroy(cs);
        return fail(SONAR_E_NOMEM, "host allocation failed");
    }
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = batch_launch_all(b, cs);
        e = hipStreamEndCapture(cs, &g->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return fail(SONAR_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    }
    *out = g;
    return SONAR_OK;
}

sonar_status sonar_graph_launch(sonar_graph *g, sonar_stream stream)
{
    if (!g || !g->exec) return fail(SONAR_E_INVALID, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "graph launch: %s", hipGetErrorString(e));
    return SONAR_OK;
}

void sonar_graph_free(sonar_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

static std::string tune_key(const sonar_scene *sc, const sonar_batch_plan *plan)
{
    hipDeviceProp_t prop;
    char name[128] = "unknown";
    if (hipGetDeviceProperties(&prop, sc->s.device) == hipSuccess) {
        snprintf(name, sizeof(name), "%s", prop.gcnArchName);
        for (char *c = name; *c; ++c)
            if (*c == ' ' || *c == ':') *c = '_';
    }
    char key[320];
    snprintf(key, sizeof(key), "%s/tri%lld/d%d/p%d/k%d/a%d/r%d/b%d/t%lld", name, (long long)sc->s.n_tri, sc->s.depth,
             plan->n_pings, plan->max_bounces, plan->arc, plan->retro, plan->max_bins, (long long)plan->total_tiles);
    return key;
}

sonar_status sonar_batch_autotune(const sonar_scene *sc, const sonar_batch_plan *plan, const void *dev_desc,
                                  void *ws, size_t ws_bytes, sonar_stream stream, sonar_batch_options *best,
                                  float *best_ms)
{
    g_err[0] = 0;
    if (!best || !best_ms) return fail(SONAR_E_INVALID, "best and best_ms are required");
    sonar::BatchLaunch b;
    sonar_status st = batch_launch_args(sc, plan, dev_desc, nullptr, ws, ws_bytes, &b);
    if (st != SONAR_OK) return st;
    const std::string key = tune_key(sc, plan);
    const char *cache = getenv("SONAR_AUTOTUNE_CACHE");
    if (cache && *cache) {
        FILE *f = fopen(cache, "r");
        if (f) {
            char line[512], k[400];
            int bpc, tpi, wpb;
            float ms;
            bool found = false;
            while (fgets(line, sizeof(line), f)) {
                if (sscanf(line, "%399s %d %d %d %f", k, &bpc, &tpi, &wpb, &ms) == 5 && key == k) {
                    memset(best, 0, sizeof(*best));
                    best->blocks_per_cu = bpc;
                    best->tiles_per_item = tpi;
                    best->waves_per_block = wpb;
                    *best_ms = ms;
                    found = true;
                }
            }
            fclose(f);
            if (found) return SONAR_OK;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(SONAR_E_DEVICE, "event creation failed");
    float bestv = 1e30f;
    sonar_batch_options bo;
    memset(&bo, 0, sizeof(bo));
    struct Cand { int wpb, bpc, tpi; float ms; };
    std::vector<Cand> tried;
    const bool only4 = plan->arc == 2 || plan->retro;
    const int wpbs[3] = {4, 2, 1};
    const int tpis[3] = {1, 2, 4};
    hipError_t e = hipSuccess;
    for (int wi = 0; wi < (only4 ? 1 : 3) && e == hipSuccess; ++wi) {
        const int wpb = wpbs[wi];
        b.waves_per_block = wpb;
        const int occ = sonar::batch_max_blocks_per_cu(b);        // workgroups per CU at this size
        const int per_simd = (occ * wpb) / 4;                        // waves per SIMD at the limit
        for (int ws_ = 1; ws_ <= (per_simd > 0 ? per_simd : 1) && e == hipSuccess; ++ws_) {
            const int bpc = (ws_ * 4) / wpb > 0 ? (ws_ * 4) / wpb : 1;
            for (int ti = 0; ti < 3 && e == hipSuccess; ++ti) {
                b.blocks_per_cu = bpc;
                b.tiles_per_item = tpis[ti];
                e = sonar::launch_ping_batch(b, s);   // warm-up
                float total = 0.f;
                for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
                    e = hipEventRecord(e0, s);
                    if (e == hipSuccess) e = sonar::launch_ping_batch(b, s);
                    if (e == hipSuccess) e = hipEventRecord(e1, s);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    total += ms;
                }
                if (e != hipSuccess) break;
                const float ms = total / 3.f;
                tried.push_back(Cand{wpb, bpc, tpis[ti], ms});
                if (ms < bestv) {
                    bestv = ms;
                    bo.blocks_per_cu = bpc;
                    bo.tiles_per_item = tpis[ti];
                    bo.waves_per_block = wpb;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(SONAR_E_DEVICE, "autotune run: %s", hipGetErrorString(e));
    *best = bo;
    *best_ms = bestv;
    if (cache && *cache) {
        FILE *f = fopen(cache, "a");
        if (f) {
            for (const Cand &c : tried)
                fprintf(f, "cand:%s %d %d %d %.6f\n", key.c_str(), c.bpc, c.tpi, c.wpb, c.ms);
            fprintf(f, "%s %d %d %d %.6f\n", key.c_str(), bo.blocks_per_cu, bo.tiles_per_item, bo.waves_per_block, bestv);
            fclose(f);
        }
    }
    return SONAR_OK;
}

int64_t sonar_surrogate_param_count(void) { return sonar::surrogate_param_count(); }

sonar_status sonar_surrogate_create(int64_t max_rows, int32_t n_bins, double r_min, double r_max, int32_t smooth,
                                    sonar_surrogate **out)
{
    g_err[0] = 0;
    if (!out) return fail(SONAR_E_INVALID, "out is NULL");
    *out = nullptr;
    if (max_rows < 64 || max_rows % 64 != 0 || max_rows > ((int64_t)1 << 26))
        return fail(SONAR_E_INVALID, "max_rows must be a positive multiple of 64, at most 2^26");
    if (n_bins < 64 || n_bins > 2048) return fail(SONAR_E_INVALID, "n_bins must be in [64, 2048]");
    if (!(r_min >= 0) || !(r_max > r_min) || !isfinite(r_max)) return fail(SONAR_E_INVALID, "need 0 <= r_min < r_max");
    if (smooth < 1 || smooth > n_bins) return fail(SONAR_E_INVALID, "smooth must be in [1, n_bins]");
    sonar_surrogate *h = new (std::nothrow) sonar_surrogate();
    if (!h) return fail(SONAR_E_NOMEM, "host allocation failed");
    hipError_t e = sonar::surrogate_create(max_rows, n_bins, (float)r_min, (float)r_max, smooth, &h->s);
    if (e != hipSuccess) {
        delete h;
        return fail(e == hipErrorOutOfMemory ? SONAR_E_NOMEM : SONAR_E_DEVICE, "surrogate: %s", hipGetErrorString(e));
    }
    *out = h;
    return SONAR_OK;
}

void sonar_surrogate_free(sonar_surrogate *h)
{
    if (!h) return;
    sonar::surrogate_free(h->s);
    delete h;
}

sonar_status sonar_surrogate_set_state(sonar_surrogate *h, const float *params, const float *m, const float *v,
                                       int64_t step)
{
    if (!h || !params) return fail(SONAR_E_INVALID, "surrogate and params are required");
    if ((m == nullptr) != (v == nullptr)) return fail(SONAR_E_INVALID, "give both Adam moments or neither");
    if (step < 0) return fail(SONAR_E_INVALID, "step must be >= 0");
    hipError_t e = sonar::surrogate_set_state(h->s, params, m, v, step);
    return e == hipSuccess ? SONAR_OK : fail(SONAR_E_DEVICE, "set_state: %s", hipGetErrorString(e));
}

sonar_status sonar_surrogate_get_state(const sonar_surrogate *h, float *params, float *m, float *v, int64_t *step)
{
    if (!h) return fail(SONAR_E_INVALID, "surrogate is NULL");
    hipError_t e = sonar::surrogate_get_state(h->s, params, m, v, step);
    return e == hipSuccess ? SONAR_OK : fail(SONAR_E_DEVICE, "get_state: %s", hipGetErrorString(e));
}

sonar_status sonar_surrogate_set_norm(sonar_surrogate *h, const float *mean, const float *sd)
{
    if (!h || !mean || !sd) return fail(SONAR_E_INVALID, "surrogate, mean and std are required");
    for (int j = 0; j < 64; ++j)
        if (!isfinite(mean[j]) || !(sd[j] > 0.f) || !isfinite(sd[j]))
            return fail(SONAR_E_INVALID, "std must be positive and finite");
    hipError_t e = sonar::surrogate_set_norm(h->s, mean, sd);
    return e == hipSuccess ? SONAR_OK : fail(SONAR_E_DEVICE, "set_norm: %s", hipGetErrorString(e));
}

sonar_status sonar_surrogate_set_loss_weights(sonar_surrogate *h, const float *w)
{
    if (!h) return fail(SONAR_E_INVALID, "surrogate is NULL");
    if (w)
        for (int j = 0; j < 64; ++j)
            if (!(w[j] >= 0.f) || !isfinite(w[j])) return fail(SONAR_E_INVALID, "loss weights must be finite and >= 0");
    hipError_t e = sonar::surrogate_set_loss_weights(h->s, w);
    return e == hipSuccess ? SONAR_OK : fail(SONAR_E_DEVICE, "set_loss_weights: %s", hipGetErrorString(e));
}

static sonar_status check_gbuf(const sonar_surrogate *h, const float *g, int32_t n, int32_t H, int32_t W)
{
    if (!h || !g) return fail(SONAR_E_INVALID, "surrogate and gbuffer are required");
    if (((uintptr_t)g & 15) != 0) return fail(SONAR_E_INVALID, "gbuffer must be 16-byte aligned");
    if (n < 1 || H < 1 || W < 1) return fail(SONAR_E_INVALID, "n_img, h, w must be >= 1");
    const int64_t rows = (int64_t)n * H * W;
    if (rows % 64 != 0) return fail(SONAR_E_INVALID, "n_img * h * w must be a multiple of 64");
    if (rows > sonar::surrogate_max_rows(h->s)) return fail(SONAR_E_INVALID, "more rows than max_rows");
    return SONAR_OK;
}

sonar_status sonar_surrogate_geometry(const sonar_params *p, const sonar_pose *q, float block[16])
{
    g_err[0] = 0;
    if (!p || !q || !block) return fail(SONAR_E_INVALID, "params, pose and block are required");
    if (p->grid_mode != 0) return fail(SONAR_E_UNSUPPORTED, "the surrogate's beams are cell-centred (grid_mode 0)");
    if (!(p->hfov > 0.0) || !(p->vfov > 0.0)) return fail(SONAR_E_INVALID, "fields of view must be positive");
    for (int i = 0; i < 3; ++i) block[i] = (float)q->position[i];
    for (int i = 0; i < 9; ++i) block[3 + i] = (float)q->rot[i];
    block[12] = (float)p->hfov;
    block[13] = (float)p->vfov;
    block[14] = block[15] = 0.f;
    return SONAR_OK;
}

sonar_status sonar_surrogate_forward(sonar_surrogate *h, const float *g, const float *geo, int32_t n, int32_t H,
                                     int32_t W, float *coef, sonar_stream stream)
{
    g_err[0] = 0;
    sonar_status st = check_gbuf(h, g, n, H, W);
    if (st != SONAR_OK) return st;
    if (!coef || !geo) return fail(SONAR_E_INVALID, "coef and geometry are required");
    hipError_t e = sonar::surrogate_forward(h->s, g, geo, n, H, W, coef, (hipStream_t)stream);
    return e == hipSuccess ? SONAR_OK : fail(SONAR_E_DEVICE, "forward: %s", hipGetErrorString(e));
}

sonar_status sonar_surrogate_train_step(sonar_surrogate *h, const float *g, const float *geo, int32_t n, int32_t H,
                                        int32_t W, const float *target, float lr, float *dev_loss, sonar_stream stream)
{
    g_err[0] = 0;
    sonar_status st = check_gbuf(h, g, n, H, W);
    if (st != SONAR_OK) return st;
    if (!target || !dev_loss || !geo) return fail(SONAR_E_INVALID, "geometry, target and dev_loss are required");
    if (!(lr >= 0.f) || !isfinite(lr)) return fail(SONAR_E_INVALID, "lr must be finite and >= 0");
    hipError_t e = sonar::surrogate_train_step(h->s, g, geo, n, H, W, target, lr, dev_loss, (hipStream_t)stream);
    return e == hipSuccess ? SONAR_OK : fail(SONAR_E_DEVICE, "train_step: %s", hipGetErrorString(e));
}

sonar_status sonar_surrogate_gradient(sonar_surrogate *h, const float *g, const float *geo, int32_t n, int32_t H,
                                      int32_t W, const float *target, float *dev_grad, float *dev_loss,
                                      sonar_stream stream)
{
    g_err[0] = 0;
    sonar_status st = check_gbuf(h, g, n, H, W);
    if (st != SONAR_OK) return st;
    if (!target || !dev_grad || !dev_loss || !geo)
        return fail(SONAR_E_INVALID, "geometry, target, dev_grad and dev_loss are required");
    hipError_t e = sonar::surrogate_gradient(h->s, g, geo, n, H, W, target, dev_grad, dev_loss, (hipStream_t)stream);
    return e == hipSuccess ? SONAR_OK : fail(SONAR_E_DEVICE, "gradient: %s", hipGetErrorString(e));
}

sonar_status sonar_surrogate_target(const sonar_surrogate *h, const float *im, const float *gbuffer, int64_t rows,
                                    int32_t standardize, float *coef, sonar_stream stream)
{
    g_err[0] = 0;
    if (!h || !im || !gbuffer || !coef) return fail(SONAR_E_INVALID, "surrogate, im, gbuffer and coef are required");
    if (rows < 1 || rows > sonar::surrogate_max_rows(h->s)) return fail(SONAR_E_INVALID, "rows must be in [1, max_rows]");
    hipError_t e = sonar::surrogate_target_coef(h->s, im, gbuffer, rows, standardize ? 1 : 0, coef,
                                                (hipStream_t)stream);
    return e == hipSuccess ? SONAR_OK : fail(SONAR_E_DEVICE, "target: %s", hipGetErrorString(e));
}

sonar_status sonar_surrogate_moments(sonar_surrogate *h, const float *coef, int64_t rows, double *sum, double *sq,
                                     sonar_stream stream)
{
    g_err[0] = 0;
    if (!h || !coef || !sum || !sq) return fail(SONAR_E_INVALID, "surrogate, coef, sum and sum_sq are required");
    if (rows < 1 || rows > sonar::surrogate_max_rows(h->s)) return fail(SONAR_E_INVALID, "rows must be in [1, max_rows]");
    hipError_t e = sonar::surrogate_coef_moments(h->s, coef, rows, sum, sq, (hipStream_t)stream);
    return e == hipSuccess ? SONAR_OK : fail(SONAR_E_DEVICE, "moments: %s", hipGetErrorString(e));
}

sonar_status sonar_surrogate_profile(const sonar_surrogate *h, const float *coef, const float *i1, const float *im,
                                     const float *gbuffer, int64_t rows, float *profile, float *err,
                                     sonar_stream stream)
{
    g_err[0] = 0;
    if (!h || !coef || !i1 || !gbuffer) return fail(SONAR_E_INVALID, "surrogate, coef, i1 and gbuffer are required");
    if (rows < 1 || rows > sonar::surrogate_max_rows(h->s)) return fail(SONAR_E_INVALID, "rows must be in [1, max_rows]");
    if (err && !im) return fail(SONAR_E_INVALID, "errors need the multi-bounce channel im");
    hipError_t e = sonar::surrogate_profile_errors(h->s, coef, i1, im, gbuffer, rows, err, profile,
                                                   (hipStream_t)stream);
    return e == hipSuccess ? SONAR_OK : fail(SONAR_E_DEVICE, "profile: %s", hipGetErrorString(e));
}

sonar_status sonar_device_status(const sonar_scene *sc, sonar_stream stream)
{
    if (!sc) return fail(SONAR_E_INVALID, "scene is NULL");
    int h = 0;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&h, sc->s.status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(SONAR_E_DEVICE, "status read failed");
    if (h) {
        int zero = 0;
        (void)hipMemcpyAsync(sc->s.status, &zero, sizeof(int), hipMemcpyHostToDevice, s);
        (void)hipStreamSynchronize(s);
    }
    if (h & sonar::ST_STACK) return fail(SONAR_E_STACK, "a traversal overflowed its stack; those rays were misses");
    if (h & sonar::ST_RX_FULL) return fail(SONAR_E_DEVICE, "receive-binning list full: returns were dropped");
    return SONAR_OK;
}

}  // extern "C"
