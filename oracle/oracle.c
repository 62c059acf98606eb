/*
 * Plain FP64 CPU oracle of the volumetric sonar echo model.
 *
 * TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
 * baseline load this library; the product path never does. It shares no code,
 * header, table or helper with the HIP library.
 *
 * What it follows in the paper:
 *   Sec. III, Eq. (1)-(3)  sampling-grid counts N_range, N_H, N_V, and the
 *                          LiDAR firing grid N_L = N_V + 1, N_R = N_H + 1.
 *   Sec. II-A              the sensor is volumetric: the aperture is split in
 *                          azimuth and elevation and the output is an
 *                          azimuth x elevation x range distribution of
 *                          backscatter; rays bend by Snell's law in a
 *                          sound-speed field.
 *   Sec. II-B              each intersection scatters according to incidence
 *                          angle and material coefficients; a bounded number
 *                          of secondary reflections with a tunable depth;
 *                          complex returns whose phase follows the propagation
 *                          delay, with attenuation; a beam or cell is the
 *                          complex sum over its bundle of rays.
 * Readings where the paper is silent (jitter law, spreading, absorption, the
 * multipath path model, the tie rule, CFAR constants) are stated next to the
 * code that applies them.
 *
 * Everything is brute force: every ray is tested against every triangle, so
 * the result is the definition itself. Intersection uses the plane equation
 * and signed distances to the three edges (not the Moller-Trumbore form).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_MAXK 8
#define ORC_MAXKNOTS 8

/* Beam forming options (Sec. II-B: the backscattered contribution depends on
 * the transmit-receive beam pattern).
 * ORC_BEAM_PATTERN: every contribution is weighted by the one-way amplitude
 *   pattern of the transmit beam at the launch direction times that of the
 *   receive beam at the arrival direction; the pattern of a beam is a
 *   Gaussian main lobe b = exp(-2 ln2 ((d_az / dth_h)^2 + (d_el / dth_v)^2))
 *   in the angular offsets from the beam centre, so that its one-way power
 *   is 3 dB down half a cell from the axis.
 * ORC_RX_BEAMS: a contribution of bounce >= 2 goes to the receive beam whose
 *   cell holds its arrival direction instead of the launch beam (bounce-1
 *   returns arrive along the reversed launch ray, so their beam is the launch
 *   beam). Cell-centred beams only. */
#define ORC_BEAM_PATTERN 1u
#define ORC_RX_BEAMS 2u
/* ORC_DIFFUSE_BOUNCE: the continuation after a rough facet is drawn from the
 * facet's scattering lobes instead of the mirror direction (Monte Carlo).
 * With z = SplitMix64 output c + 1 of (seed xor 0xD1B54A32D192ED03) and
 * c = (ping << 40) xor (ray << 2) xor k, u1 = (z >> 40) / 2^24,
 * u2 = ((z >> 16) mod 2^24) / 2^24, u3 = (z mod 2^16) / 2^16: the Phong lobe
 * around the mirror direction when u3 < k_s / (k_d + k_s) (cos a =
 * (1 - u1)^(1 / (n + 1))), else the cosine lobe around the facet normal
 * facing the ray (cos a = sqrt(1 - u1)); azimuth 2 pi u2 in the orthonormal
 * basis of Duff et al. (JCGT 2017) around the lobe axis. A direction that
 * does not leave the facet's lit side ends the ray. The path's amplitude
 * weight takes sqrt(rho (k_d + k_s)) (each lobe normalised and drawn with
 * its own probability). Pressure-release facets stay exact mirrors. */
#define ORC_DIFFUSE_BOUNCE 4u
/* ORC_RETRO_CHAIN: every vertex after the first also returns along its own
 * outgoing chain reversed (reciprocity: the reversed chain is the same path,
 * so it is as visible as the way out). The vertex scatters back into the
 * reversed incoming direction (departure cosine = incidence cosine, Phong
 * lobe taken toward -incident), the chain's weights apply twice (each
 * earlier vertex is met again on the way back), the path is the outgoing
 * one twice (time 2 T_out, spreading 1 / L_out^2, absorption over 2 L_out)
 * and the echo arrives along the launch ray (launch beam, transmit pattern
 * twice). */
#define ORC_RETRO_CHAIN 8u

/* ------------------------------------------------------------------------ */
/* small vector algebra                                                      */

typedef struct { double x, y, z; } v3;

static v3 mk(double x, double y, double z) { v3 r; r.x = x; r.y = y; r.z = z; return r; }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static double len(v3 a) { return sqrt(dot(a, a)); }
static v3 unit(v3 a) { return scl(a, 1.0 / len(a)); }

/* ------------------------------------------------------------------------ */
/* inputs                                                                    */

typedef struct {
    double hfov, vfov;           /* radians */
    int32_t n_h, n_v, n_r;       /* beams in azimuth / elevation, rays per beam */
    int32_t grid_mode;           /* 0 cell-centred beams, 1 LiDAR firing grid */
    int32_t jitter;              /* 1: stratified jitter, 0: stratum centres */
    int32_t n_bins;
    double r_min, r_max;
    double f0, c0, g;            /* centre frequency, c(z) = c0 + g z */
    double alpha_db;             /* absorption in dB per metre of total path */
    int32_t max_bounces;
    int32_t pad0;
    double k_d, k_s, phong_n;
    uint64_t seed;
    uint32_t ping;
    uint32_t flags;              /* ORC_BEAM_PATTERN | ORC_RX_BEAMS */
    int32_t n_knots;             /* >= 2: piecewise-linear c(z) through the knots (replaces c0, g) */
    int32_t pad2;
    double knot_z[ORC_MAXKNOTS], knot_c[ORC_MAXKNOTS];
} orc_params;

typedef struct { double pos[3]; double rot[9]; } orc_pose;   /* sensor->world, row-major */

/* Thresholds of the ambiguity flags. A ray is flagged when any of its events
 * is within these margins of a discrete decision; flagged rays are excluded
 * from index comparisons and from the masked volume. */
typedef struct {
    double graze;      /* cos(incidence) or cos(departure) below this */
    double edge_abs;   /* hit within edge_abs + edge_rel * s of a triangle edge */
    double edge_rel;
    double tie_rel;    /* a second candidate within s * (1 + tie_rel) + tie_abs */
    double tie_abs;
    double bin_frac;   /* range position within this fraction of a bin edge */
    double fov;        /* arrival direction within this angle (rad) of the FOV edge */
    double lim_rel;    /* a hit or a stop test within this relative margin of its bound */
    double self_lo, self_hi;  /* hit distances in [self_lo, self_hi] are flagged */
    double caustic;    /* layered profile: a first-arriving eigenray and another whose turning
                        * depths differ by less than this in sqrt(rise / window) */
} orc_tol;

enum {
    F_GRAZE = 1u << 0, F_EDGE = 1u << 1, F_TIE = 1u << 2, F_LIMIT = 1u << 3,
    F_SELF = 1u << 4, F_BIN = 1u << 5, F_FOV = 1u << 6, F_OCCLUDER = 1u << 7,
    F_STOP = 1u << 8, F_DEPART = 1u << 9, F_CAUSTIC = 1u << 10
};

/* Optional uniform grid over the scene (an exact candidate filter, see
 * grid_candidates): triangle i is listed in every cell that its bounding box,
 * grown by gpad[i], touches (closed intervals). */
typedef struct {
    int nx, ny, nz;
    double lo[3], h;            /* grid origin and cubic cell size */
    int64_t *start;             /* [nx ny nz + 1] CSR offsets into ids */
    int32_t *ids;
} ogrid;

typedef struct {
    int64_t nt;
    double *p;          /* [nt][9] FP32 vertices promoted exactly */
    double *nrm;        /* [nt][3] (p1 - p0) x (p2 - p0) */
    double *rho, *phi;
    uint8_t *mat;
    double zabs_max;    /* max |z| over all vertices */
    ogrid *grid;        /* NULL: every query loops over all triangles */
} oscene;

static const double EPS_SELF = 1e-4;   /* minimum hit distance, metres */

/* ------------------------------------------------------------------------ */
/* scene                                                                     */

void *orc_scene_new(const float *v, int64_t nv, const int32_t *idx, int64_t nt,
                    const float *rho, const float *phi, const uint8_t *mat)
{
    (void)nv;
    oscene *s = (oscene *)calloc(1, sizeof(oscene));
    s->nt = nt;
    s->p = (double *)malloc(sizeof(double) * 9 * (size_t)nt);
    s->nrm = (double *)malloc(sizeof(double) * 3 * (size_t)nt);
    s->rho = (double *)malloc(sizeof(double) * (size_t)nt);
    s->phi = (double *)malloc(sizeof(double) * (size_t)nt);
    s->mat = (uint8_t *)malloc((size_t)nt);
    double zmax = 0.0;
    for (int64_t i = 0; i < nt; ++i) {
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a) {
                double w = (double)v[3 * (int64_t)idx[3 * i + c] + a];
                s->p[9 * i + 3 * c + a] = w;
                if (a == 2 && fabs(w) > zmax) zmax = fabs(w);
            }
        v3 p0 = mk(s->p[9 * i], s->p[9 * i + 1], s->p[9 * i + 2]);
        v3 p1 = mk(s->p[9 * i + 3], s->p[9 * i + 4], s->p[9 * i + 5]);
        v3 p2 = mk(s->p[9 * i + 6], s->p[9 * i + 7], s->p[9 * i + 8]);
        v3 n = cross(sub(p1, p0), sub(p2, p0));
        s->nrm[3 * i] = n.x; s->nrm[3 * i + 1] = n.y; s->nrm[3 * i + 2] = n.z;
        s->rho[i] = rho[i];
        s->phi[i] = phi[i];
        s->mat[i] = mat[i];
    }
    s->zabs_max = zmax;
    return s;
}

void orc_scene_free(void *h)
{
    oscene *s = (oscene *)h;
    if (!s) return;
    if (s->grid) { free(s->grid->start); free(s->grid->ids); free(s->grid); }
    free(s->p); free(s->nrm); free(s->rho); free(s->phi); free(s->mat); free(s);
}

static v3 tri_vertex(const oscene *s, int64_t i, int c)
{
    const double *q = s->p + 9 * i + 3 * c;
    return mk(q[0], q[1], q[2]);
}

static v3 tri_normal(const oscene *s, int64_t i)
{
    return mk(s->nrm[3 * i], s->nrm[3 * i + 1], s->nrm[3 * i + 2]);
}

/* Signed distance (metres) from a point of the triangle's plane to the nearest
 * edge line: positive inside, negative outside. */
static double edge_distance(const oscene *s, int64_t i, v3 P)
{
    v3 n = tri_normal(s, i);
    double nl = len(n);
    double best = 1e300;
    for (int e = 0; e < 3; ++e) {
        v3 a = tri_vertex(s, i, e), b = tri_vertex(s, i, (e + 1) % 3);
        v3 ed = sub(b, a);
        double el = len(ed);
        double d = dot(cross(n, ed), sub(P, a)) / (nl * el);
        if (d < best) best = d;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Exact candidate filter (a uniform grid, Amanatides and Woo 1987).         */
/*                                                                           */
/* A triangle changes a query's result or flags only through a plane root s  */
/* on the queried path piece whose point X(s) has edge_distance > -dl, with  */
/* dl = edge_abs + edge_rel * s (nearest_hit_from, blocked_piece). X then    */
/* lies in the triangle grown by dl across each edge, inside the triangle's  */
/* bounding box grown by dl / sin(a / 2), a its smallest angle. The piece    */
/* lies within its sagitta of the chord between its ends, and the cells the  */
/* chord passes are walked one by one. Triangles are binned with their box   */
/* grown by GRID_DL / sin(a / 2) + GRID_FAT, so a query is exact while its   */
/* dl stays below GRID_DL and its sagitta below GRID_FAT - 1e-6 (rounding of */
/* the walk is far below the remaining millimetres); other queries loop over */
/* all triangles. Candidates are visited in increasing index, the order of   */
/* the full loop, so ties resolve identically. Triangles with no area have   */
/* no plane roots and are not binned; near-slivers whose grown box would    */
/* span the scene are tested by every query.                                */

#define GRID_DL 1e-3
#define GRID_FAT 1e-2

static int cmp_i32(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Grid padding of triangle i, or -1 for a triangle without area. */
static double grid_pad(const oscene *s, int64_t i)
{
    v3 n = tri_normal(s, i);
    if (dot(n, n) == 0.0) return -1.0;
    double smin = 1.0;
    for (int c = 0; c < 3; ++c) {
        v3 a = sub(tri_vertex(s, i, (c + 1) % 3), tri_vertex(s, i, c));
        v3 b = sub(tri_vertex(s, i, (c + 2) % 3), tri_vertex(s, i, c));
        double cs = dot(a, b) / (len(a) * len(b));
        double sh = sqrt(0.5 * (1.0 - cs));        /* sin of half the vertex angle */
        if (sh < smin) smin = sh;
    }
    if (!(smin > 0.0)) return 1e300;
    return GRID_DL / smin + GRID_FAT + 1e-6;
}

/* Builds the grid with about `cells_per_tri` cells per triangle. */
void orc_scene_build_grid(void *hs, double cells_per_tri)
{
    oscene *S = (oscene *)hs;
    if (S->grid) { free(S->grid->start); free(S->grid->ids); free(S->grid); S->grid = NULL; }
    const int64_t nt = S->nt;
    double *bx = (double *)malloc(sizeof(double) * 6 * (size_t)nt);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < nt; ++i) {
        double *b = bx + 6 * i;
        b[0] = 1.0; b[3] = -1.0;                   /* empty: not binned */
        if (grid_pad(S, i) < 0.0) continue;
        for (int a = 0; a < 3; ++a) {
            double l = S->p[9 * i + a], h = l;
            for (int c = 1; c < 3; ++c) {
                double w = S->p[9 * i + 3 * c + a];
                if (w < l) l = w;
                if (w > h) h = w;
            }
            b[a] = l; b[3 + a] = h;
            if (l < lo[a]) lo[a] = l;
            if (h > hi[a]) hi[a] = h;
        }
    }
    /* extent of the scene without padding */
    double span = 0.0;
    for (int a = 0; a < 3; ++a) if (hi[a] - lo[a] > span) span = hi[a] - lo[a];
    ogrid *G = (ogrid *)calloc(1, sizeof(ogrid));
    const double big = span + 1.0;                 /* a grown box wider than this spans the grid */
    double glo[3], ghi[3];
    for (int a = 0; a < 3; ++a) { glo[a] = lo[a] - GRID_FAT - 1.0; ghi[a] = hi[a] + GRID_FAT + 1.0; }
    double vol = (ghi[0] - glo[0]) * (ghi[1] - glo[1]) * (ghi[2] - glo[2]);
    double hcell = cbrt(vol / (cells_per_tri * (double)(nt > 0 ? nt : 1)));
    int n[3];
    for (int a = 0; a < 3; ++a) {
        double c = ceil((ghi[a] - glo[a]) / hcell);
        if (c < 1) c = 1;
        if (c > 2048) c = 2048;
        n[a] = (int)c;
    }
    /* the cell size must cover the extent with the clamped counts */
    for (int a = 0; a < 3; ++a) {
        double need = (ghi[a] - glo[a]) / n[a];
        if (need > hcell) hcell = need;
    }
    G->nx = n[0]; G->ny = n[1]; G->nz = n[2];
    for (int a = 0; a < 3; ++a) G->lo[a] = glo[a];
    G->h = hcell;
    const int64_t ncell = (int64_t)n[0] * n[1] * n[2];
    G->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    /* two passes over the triangles: counts, then ids (in increasing index within every cell) */
    for (int pass = 0; pass < 2; ++pass) {
        int64_t *fill = NULL;
        if (pass == 1) {
            for (int64_t c = 0; c < ncell; ++c) G->start[c + 1] += G->start[c];
            G->ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(G->start[ncell] > 0 ? G->start[ncell] : 1));
            fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
            memcpy(fill, G->start, sizeof(int64_t) * (size_t)ncell);
        }
        for (int64_t i = 0; i < nt; ++i) {
            const double *b = bx + 6 * i;
            if (b[0] > b[3]) continue;
            double pad = grid_pad(S, i);
            if (pad > big) pad = big;              /* a near-sliver: every cell */
            int c0[3], c1[3];
            for (int a = 0; a < 3; ++a) {
                double l = floor((b[a] - pad - glo[a]) / hcell), h = floor((b[3 + a] + pad - glo[a]) / hcell);
                if (l < 0) l = 0;
                if (h > n[a] - 1) h = n[a] - 1;
                c0[a] = (int)l; c1[a] = (int)h;
            }
            for (int z = c0[2]; z <= c1[2]; ++z)
                for (int y = c0[1]; y <= c1[1]; ++y)
                    for (int x = c0[0]; x <= c1[0]; ++x) {
                        int64_t c = ((int64_t)z * n[1] + y) * n[0] + x;
                        if (pass == 0) ++G->start[c + 1];
                        else G->ids[fill[c]++] = (int32_t)i;
                    }
        }
        free(fill);
    }
    free(bx);
    S->grid = G;
}

/* Cells in the grid, listed triangle entries, cell size. */
void orc_scene_grid_info(const void *hs, double out[3])
{
    const oscene *S = (const oscene *)hs;
    out[0] = out[1] = out[2] = 0.0;
    if (!S->grid) return;
    const ogrid *G = S->grid;
    const int64_t nc = (int64_t)G->nx * G->ny * G->nz;
    out[0] = (double)nc;
    out[1] = (double)G->start[nc];
    out[2] = G->h;
}

/* ------------------------------------------------------------------------ */
/* Sec. III, Eq. (1)-(3): grid counts. floor() of a quotient that is an       */
/* integer in exact arithmetic is taken with a 1e-9 guard against rounding.  */

void orc_grid_counts(double hfov, double vfov, double dth_h, double dth_v, double r_min,
                     double r_max, double dr, int32_t out[6])
{
    out[0] = (int32_t)floor((r_max - r_min) / dr + 1e-9);    /* N_range */
    out[1] = (int32_t)floor(hfov / dth_h + 1e-9);            /* N_H */
    out[2] = (int32_t)floor(vfov / dth_v + 1e-9);            /* N_V */
    out[3] = out[2] + 1;                                     /* N_L: elevation rows */
    out[4] = out[1] + 1;                                     /* N_R: rays per row */
    out[5] = out[3] * out[4];                                /* N_E: emitters */
}

/* ------------------------------------------------------------------------ */
/* Ray generation. Jitter uniforms are the (counter + 1)-th output of the     */
/* SplitMix64 generator (Steele, Lea and Flood, OOPSLA 2014) seeded with      */
/* `seed`; the counter packs (ping, beam, ray).                              */

static uint64_t splitmix_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64_nth(uint64_t seed, uint64_t n)
{
    return splitmix_mix(seed + n * 0x9E3779B97F4A7C15ULL);
}

void orc_jitter(uint64_t seed, uint32_t ping, uint32_t beam, uint32_t ray, double out[2])
{
    uint64_t ctr = ((uint64_t)ping << 40) ^ ((uint64_t)beam << 8) ^ (uint64_t)ray;
    uint64_t z = orc_splitmix64_nth(seed, ctr + 1);
    out[0] = (double)(z >> 40) * (1.0 / 16777216.0);
    out[1] = (double)((z >> 16) & 0xFFFFFFu) * (1.0 / 16777216.0);
}

static void strata(int n_r, int *na, int *ne)
{
    int lg = 0;
    while ((1 << (lg + 1)) <= n_r) ++lg;
    *ne = 1 << (lg / 2);
    *na = n_r / *ne;
}

static int beams_h(const orc_params *P) { return P->grid_mode == 1 ? P->n_h + 1 : P->n_h; }


static v3 sensor_to_world(const orc_pose *Q, v3 a)
{
    const double *R = Q->rot;
    return mk(R[0] * a.x + R[1] * a.y + R[2] * a.z,
              R[3] * a.x + R[4] * a.y + R[5] * a.z,
              R[6] * a.x + R[7] * a.y + R[8] * a.z);
}

static v3 world_to_sensor(const orc_pose *Q, v3 a)
{
    const double *R = Q->rot;
    return mk(R[0] * a.x + R[3] * a.y + R[6] * a.z,
              R[1] * a.x + R[4] * a.y + R[7] * a.z,
              R[2] * a.x + R[5] * a.y + R[8] * a.z);
}

/* Azimuth/elevation of ray j of beam b. Sensor frame: x forward, y left, z up;
 * azimuth from +x toward +y, elevation toward +z; the beam index is
 * b = v * (beams per row) + h with h, v increasing with azimuth, elevation. */
static void ray_angles(const orc_params *P, int b, int j, double *az, double *el)
{
    int nh = beams_h(P);
    int h = b % nh, v = b / nh;
    double dh = P->hfov / P->n_h, dv = P->vfov / P->n_v;
    if (P->grid_mode == 1) {
        *az = -0.5 * P->hfov + h * dh;
        *el = -0.5 * P->vfov + v * dv;
        return;
    }
    int na, ne;
    strata(P->n_r, &na, &ne);
    int ja = j % na, je = j / na;
    double u[2] = {0.5, 0.5};
    if (P->jitter) orc_jitter(P->seed, P->ping, (uint32_t)b, (uint32_t)j, u);
    *az = -0.5 * P->hfov + (h + (ja + u[0]) / na) * dh;
    *el = -0.5 * P->vfov + (v + (je + u[1]) / ne) * dv;
}

static v3 dir_from_angles(double az, double el)
{
    return mk(cos(el) * cos(az), cos(el) * sin(az), sin(el));
}

void orc_ray(const orc_params *P, const orc_pose *Q, int32_t b, int32_t j, double out[6])
{
    double az, el;
    ray_angles(P, b, j, &az, &el);
    v3 d = sensor_to_world(Q, dir_from_angles(az, el));
    out[0] = Q->pos[0]; out[1] = Q->pos[1]; out[2] = Q->pos[2];
    out[3] = d.x; out[4] = d.y; out[5] = d.z;
}

/* ------------------------------------------------------------------------ */
/* Propagation paths. In c(z) = c0 + g z the Snell invariant cos(theta)/c is  */
/* constant, so a ray is a circle of curvature kappa = g cos(theta) / c(z)    */
/* whose centre lies on the plane c = 0 (Sec. II-A asks for ray bending by    */
/* Snell's law; the circle is its exact solution for a linear profile).      */
/* x(s) = o + d sin(ks)/k + nc (1 - cos(ks))/k, nc the in-plane unit normal.  */

typedef struct {
    int arc;            /* 0: straight line */
    v3 o, d, nc;
    double kappa;
} opath;

static opath make_path_gc(double g, double c0, v3 o, v3 d)
{
    opath r;
    r.o = o; r.d = d; r.arc = 0; r.kappa = 0.0; r.nc = mk(0, 0, 0);
    double dh = hypot(d.x, d.y);
    if (g == 0.0 || dh == 0.0) return r;
    double c = c0 + g * o.z;
    r.arc = 1;
    r.kappa = g * dh / c;
    r.nc = mk(d.z * d.x / dh, d.z * d.y / dh, -dh);
    return r;
}

static opath make_path(const orc_params *P, v3 o, v3 d) { return make_path_gc(P->g, P->c0, o, d); }

static v3 path_point(const opath *p, double s)
{
    if (!p->arc) return add(p->o, scl(p->d, s));
    double u = p->kappa * s;
    double sh = sin(0.5 * u);
    return add(p->o, add(scl(p->d, sin(u) / p->kappa), scl(p->nc, 2.0 * sh * sh / p->kappa)));
}

static v3 path_tangent(const opath *p, double s)
{
    if (!p->arc) return p->d;
    double u = p->kappa * s;
    return add(scl(p->d, cos(u)), scl(p->nc, sin(u)));
}

/* One-way travel time along the path from s = 0 to s. For the arc, the
 * integral of ds / c along a circle of a linear profile is
 * (atanh(sin th0) - atanh(sin th1)) / g (Jensen et al., Computational Ocean
 * Acoustics, ch. 3), written with log1p so that no large terms cancel. */
static double path_time_gc(double g, double c0, const opath *p, double s)
{
    if (!p->arc) {
        if (g == 0.0) return s / c0;
        /* vertical ray: dt = dz / c(z) */
        double z0 = p->o.z, dz = p->d.z * s;
        return fabs(log1p(g * dz / (c0 + g * z0)) / g);
    }
    double u = p->kappa * s;
    double sh = sin(0.5 * u);
    double omc = 2.0 * sh * sh;                       /* 1 - cos u */
    double dh = hypot(p->d.x, p->d.y);
    double s0 = p->d.z;
    double ds = p->d.z * omc + dh * sin(u);           /* sin th0 - sin th1 */
    double s1 = s0 - ds;
    double dz = (p->d.z * sin(u) + p->nc.z * omc) / p->kappa;
    double lc = log1p(g * dz / (c0 + g * p->o.z));   /* ln(c1 / c0) */
    double t;
    if (s0 >= 0.0) t = log1p(ds / (1.0 + s1)) + lc;
    else t = log1p(ds / (1.0 - s0)) - lc;
    return t / g;
}

static double path_time(const orc_params *P, const opath *p, double s) { return path_time_gc(P->g, P->c0, p, s); }

/* ------------------------------------------------------------------------ */
/* Piecewise-linear sound speed (a general depth-dependent profile): layer i */
/* spans knots i..i+1 with c linear in it (the first and last layers extend  */
/* to -inf and +inf). Inside a layer the ray is that layer's circle; at a    */
/* boundary it continues with the same direction (c is continuous, so the    */
/* Snell invariant cos(theta) / c carries over) and the next curvature.      */

static int layer_count(const orc_params *P) { return P->n_knots - 1; }

static double layer_g(const orc_params *P, int i)
{
    return (P->knot_c[i + 1] - P->knot_c[i]) / (P->knot_z[i + 1] - P->knot_z[i]);
}

static double layer_c0(const orc_params *P, int i) { return P->knot_c[i] - layer_g(P, i) * P->knot_z[i]; }

static int layer_of(const orc_params *P, double z)
{
    int i = 0;
    while (i + 1 < layer_count(P) && z >= P->knot_z[i + 1]) ++i;
    return i;
}

static double profile_c(const orc_params *P, double z)
{
    int i = layer_of(P, z);
    return layer_c0(P, i) + layer_g(P, i) * z;
}

/* Arc length at which path p (in layer i) leaves the layer, and the layer it
 * enters (-1: never). The grazing angle along a circle of curvature k is
 * theta(s) = theta0 - k s, and at a boundary z_b Snell gives
 * cos(theta_b) = cos(theta0) c(z_b) / c(o); the upper boundary is reached
 * going up (theta_b > 0), the lower one going down. */
static double layer_exit(const orc_params *P, int i, const opath *p, double g, double c0, int *next,
                         uint32_t *flags)
{
    const int nl = layer_count(P);
    double best = HUGE_VAL;
    *next = -1;
    const double zb[2] = {i + 1 < nl ? P->knot_z[i + 1] : HUGE_VAL, i > 0 ? P->knot_z[i] : -HUGE_VAL};
    if (!p->arc) {
        if (p->d.z > 0.0 && zb[0] < HUGE_VAL) { best = (zb[0] - p->o.z) / p->d.z; *next = i + 1; }
        if (p->d.z < 0.0 && zb[1] > -HUGE_VAL) { best = (zb[1] - p->o.z) / p->d.z; *next = i - 1; }
        return best;
    }
    const double sz = p->d.z > 1.0 ? 1.0 : (p->d.z < -1.0 ? -1.0 : p->d.z);
    const double th0 = asin(sz), cth = hypot(p->d.x, p->d.y), co = c0 + g * p->o.z;
    for (int t = 0; t < 2; ++t) {
        if (!(fabs(zb[t]) < HUGE_VAL)) continue;
        const double C = cth * (c0 + g * zb[t]) / co;
        if (fabs(C - 1.0) < 1e-9) *flags |= F_LIMIT;      /* turning point at the boundary */
        if (C > 1.0) continue;
        const double thb = t == 0 ? acos(C) : -acos(C);
        const double s = (th0 - thb) / p->kappa;
        if (s > 1e-12 && s < best) { best = s; *next = t == 0 ? i + 1 : i - 1; }
    }
    return best;
}

static __thread int32_t *tl_cand = NULL;
static __thread int64_t tl_cap = 0;

static void cand_push(const int32_t *ids, int64_t n, int64_t *cnt)
{
    if (*cnt + n > tl_cap) {
        int64_t cap = tl_cap ? tl_cap : 4096;
        while (cap < *cnt + n) cap *= 2;
        tl_cand = (int32_t *)realloc(tl_cand, sizeof(int32_t) * (size_t)cap);
        tl_cap = cap;
    }
    memcpy(tl_cand + *cnt, ids, sizeof(int32_t) * (size_t)n);
    *cnt += n;
}

/* Candidates of the path piece p over arc length (0, hi] whose positions on
 * the whole path run up to s_end (dl grows with them): the number of
 * candidates, sorted and distinct in *out (thread-local storage, valid until
 * the next call on the thread), or -1 when the query needs the full loop. */
static int64_t grid_candidates(const oscene *S, const opath *p, double hi, double s_end, const orc_tol *T,
                               const int32_t **out)
{
    const ogrid *G = S->grid;
    if (!G) return -1;
    if (!(T->edge_abs + T->edge_rel * s_end <= GRID_DL)) return -1;
    double sag = 0.0;
    if (p->arc) {
        double u = fabs(p->kappa) * hi;
        if (!(u <= 1.0)) return -1;
        double q = sin(0.25 * u);
        sag = (2.0 * q * q / fabs(p->kappa)) * 1.01 + 1e-9;
    }
    if (!(sag <= GRID_FAT - 1e-6)) return -1;
    v3 A = p->o, B = path_point(p, hi);
    double a0[3] = {A.x, A.y, A.z}, dv[3] = {B.x - A.x, B.y - A.y, B.z - A.z};
    const int n[3] = {G->nx, G->ny, G->nz};
    /* clip t in [0, 1] to the grid box */
    double t0 = 0.0, t1 = 1.0;
    for (int a = 0; a < 3; ++a) {
        double l = G->lo[a], h = G->lo[a] + n[a] * G->h;
        if (dv[a] == 0.0) {
            if (a0[a] < l || a0[a] > h) { *out = tl_cand; return 0; }
            continue;
        }
        double ta = (l - a0[a]) / dv[a], tb = (h - a0[a]) / dv[a];
        if (ta > tb) { double w = ta; ta = tb; tb = w; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    int64_t cnt = 0;
    if (t0 <= t1) {
        int c[3], step[3];
        double tmax[3], tdel[3];
        for (int a = 0; a < 3; ++a) {
            double x = a0[a] + t0 * dv[a];
            int ci = (int)floor((x - G->lo[a]) / G->h);
            if (ci < 0) ci = 0;
            if (ci > n[a] - 1) ci = n[a] - 1;
            c[a] = ci;
            if (dv[a] > 0.0) {
                step[a] = 1;
                tmax[a] = (G->lo[a] + (ci + 1) * G->h - a0[a]) / dv[a];
                tdel[a] = G->h / dv[a];
            } else if (dv[a] < 0.0) {
                step[a] = -1;
                tmax[a] = (G->lo[a] + ci * G->h - a0[a]) / dv[a];
                tdel[a] = -G->h / dv[a];
            } else {
                step[a] = 0;
                tmax[a] = 1e300;
                tdel[a] = 1e300;
            }
        }
        for (;;) {
            int64_t cell = ((int64_t)c[2] * n[1] + c[1]) * n[0] + c[0];
            cand_push(G->ids + G->start[cell], G->start[cell + 1] - G->start[cell], &cnt);
            int a = 0;
            if (tmax[1] < tmax[a]) a = 1;
            if (tmax[2] < tmax[a]) a = 2;
            if (tmax[a] > t1) break;
            c[a] += step[a];
            if (c[a] < 0 || c[a] >= n[a]) break;
            tmax[a] += tdel[a];
        }
    }
    if (cnt > 1) {
        qsort(tl_cand, (size_t)cnt, sizeof(int32_t), cmp_i32);
        int64_t m = 1;
        for (int64_t k = 1; k < cnt; ++k)
            if (tl_cand[k] != tl_cand[m - 1]) tl_cand[m++] = tl_cand[k];
        cnt = m;
    }
    *out = tl_cand;
    return cnt;
}

/* Roots s in (0, hi] of the path meeting the plane of triangle i. */
static int plane_roots(const oscene *S, int64_t i, const opath *p, double hi, double r[2])
{
    v3 n = tri_normal(S, i);
    v3 p0 = tri_vertex(S, i, 0);
    double a = dot(n, sub(p->o, p0));
    double b = dot(n, p->d);
    if (!p->arc) {
        if (b == 0.0) return 0;
        double s = -a / b;
        if (s > 0.0 && s <= hi) { r[0] = s; return 1; }
        return 0;
    }
    /* a + (b sin u + c (1 - cos u)) / k = 0 with u = k s. The half-angle
     * substitution w = tan(u / 2) (sin u = 2w / (1 + w^2), 1 - cos u =
     * 2w^2 / (1 + w^2)) turns it exactly into the quadratic
     * (2c + a k) w^2 + 2b w + a k = 0, solved in the cancellation-free form;
     * then u = 2 atan(w). As k -> 0 the small root tends to s = -a / b. */
    double c = dot(n, p->nc);
    double k = p->kappa;
    double qa = 2.0 * c + a * k, qb = 2.0 * b, qc = a * k;
    double disc = qb * qb - 4.0 * qa * qc;
    if (disc < 0.0) return 0;
    double sq = sqrt(disc);
    double q = -0.5 * (qb + (qb >= 0.0 ? sq : -sq));
    double wr[2];
    int nw = 0;
    if (qa != 0.0) wr[nw++] = q / qa;
    if (q != 0.0) wr[nw++] = qc / q;
    int m = 0;
    for (int t = 0; t < nw; ++t) {
        double s = 2.0 * atan(wr[t]) / k;
        if (s > 0.0 && s <= hi) r[m++] = s;
    }
    if (m == 2 && r[1] < r[0]) { double w = r[0]; r[0] = r[1]; r[1] = w; }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Nearest hit by brute force. Valid: triangle != prev, eps < s <= s_lim and  */
/* the point lies inside the closed triangle. Tie rule: smallest s, then the */
/* lowest triangle index. Flags mark candidates that a finite-precision      */
/* search could resolve differently.                                         */

typedef struct {
    int64_t tri;
    double s;
    uint32_t flags;
} ohit;

static ohit nearest_hit_from(const oscene *S, const opath *p, int64_t prev, double s_min, double s_lim,
                             const orc_tol *T);

static ohit nearest_hit(const oscene *S, const opath *p, int64_t prev, double s_lim, const orc_tol *T)
{
    return nearest_hit_from(S, p, prev, EPS_SELF, s_lim, T);
}

static ohit nearest_hit_from(const oscene *S, const opath *p, int64_t prev, double s_min, double s_lim,
                             const orc_tol *T)
{
    ohit h;
    h.tri = -1; h.s = 0.0; h.flags = 0;
    double hi = s_lim * (1.0 + T->lim_rel) + 1e-9;
    double best = 1e300;
    double near1 = 1e300, near2 = 1e300;   /* the two nearest near-candidates */
    int64_t near1_i = -1;
    const int32_t *cand;
    const int64_t nc = grid_candidates(S, p, hi, hi, T, &cand);
    const int64_t n_loop = nc >= 0 ? nc : S->nt;
    for (int64_t c = 0; c < n_loop; ++c) {
        const int64_t i = nc >= 0 ? (int64_t)cand[c] : c;
        if (i == prev) continue;
        double r[2];
        int m = plane_roots(S, i, p, hi, r);
        for (int t = 0; t < m; ++t) {
            double s = r[t];
            v3 X = path_point(p, s);
            double de = edge_distance(S, i, X);
            if (s > s_min && s <= s_lim && de >= 0.0 && s < best) {
                best = s;
                h.tri = i;
            }
            double dl = T->edge_abs + T->edge_rel * s;
            if (de > -dl && s >= T->self_lo) {
                if (s < near1) { near2 = near1; near1 = s; near1_i = i; }
                else if (s < near2) near2 = s;
            }
        }
    }
    if (h.tri >= 0) {
        h.s = best;
        v3 X = path_point(p, best);
        double de = edge_distance(S, h.tri, X);
        if (de < T->edge_abs + T->edge_rel * best) h.flags |= F_EDGE;
        double other = (near1_i == h.tri) ? near2 : near1;
        if (other <= best * (1.0 + T->tie_rel) + T->tie_abs) h.flags |= F_TIE;
        if (best >= s_lim * (1.0 - T->lim_rel)) h.flags |= F_LIMIT;
        if (best <= T->self_hi) h.flags |= F_SELF;
    } else {
        if (near1 <= hi) h.flags |= F_TIE;
    }
    return h;
}

/* Any hit of piece p of a path of total length L, the piece starting at arc
 * length s0 and running for len, other than `skip`: a hit at path length s
 * counts on (eps, L - eps); occluders near an edge or near either end of the
 * path are flagged. Returns 1 when the piece is blocked. */
static int blocked_piece(const oscene *S, const opath *p, int64_t skip, double s0, double len, double L,
                         const orc_tol *T, uint32_t *flags)
{
    int hit = 0;
    const int32_t *cand;
    const int64_t nc = grid_candidates(S, p, len, s0 + len, T, &cand);
    const int64_t n_loop = nc >= 0 ? nc : S->nt;
    for (int64_t c = 0; c < n_loop; ++c) {
        const int64_t i = nc >= 0 ? (int64_t)cand[c] : c;
        if (i == skip) continue;
        double r[2];
        int m = plane_roots(S, i, p, len, r);
        for (int t = 0; t < m; ++t) {
            double s = s0 + r[t];
            v3 X = path_point(p, r[t]);
            double de = edge_distance(S, i, X);
            double dl = T->edge_abs + T->edge_rel * s;
            int inside_range = (s > EPS_SELF && s < L - EPS_SELF);
            if (inside_range && de >= 0.0) hit = 1;
            if (de > -dl) {
                if (inside_range && de < dl) *flags |= F_OCCLUDER;
                if (s >= T->self_lo && s <= T->self_hi) *flags |= F_OCCLUDER;
                if (s >= L - T->self_hi && s <= L - T->self_lo) *flags |= F_OCCLUDER;
            }
        }
    }
    return hit;
}

/* Any hit on (eps, L - eps) of a one-piece path other than `skip`. */
static int blocked(const oscene *S, const opath *p, int64_t skip, double L, const orc_tol *T, uint32_t *flags)
{
    return blocked_piece(S, p, skip, 0.0, L, L, T, flags);
}

/* ------------------------------------------------------------------------ */
/* Connection from a scattering point P back to the sensor at Sp. Straight    */
/* segment when g = 0; otherwise the eigenray: the circle through both points */
/* with its centre on the plane c = 0, in their vertical plane.              */

typedef struct {
    double L, T;        /* arc length and one-way time P -> S */
    v3 w_out;           /* unit departure direction at P */
    v3 arrive;          /* unit direction of travel at S */
    opath path;         /* the path from P */
} oconn;

static oconn connection(const orc_params *P, v3 Pp, v3 Sp)
{
    oconn c;
    v3 dv = sub(Sp, Pp);
    double D = hypot(dv.x, dv.y);
    if (P->g == 0.0 || D == 0.0) {
        c.L = len(dv);
        c.w_out = scl(dv, 1.0 / c.L);
        c.arrive = c.w_out;
        if (P->g == 0.0) c.T = c.L / P->c0;
        else c.T = fabs(log1p(P->g * dv.z / (P->c0 + P->g * Pp.z)) / P->g);
        c.path = make_path(P, Pp, c.w_out);
        return c;
    }
    /* Work in a frame where g > 0: z' = sg z. The centre plane is z' = -c0/|g|. */
    double sg = P->g > 0 ? 1.0 : -1.0;
    double ag = fabs(P->g);
    double zs = -P->c0 / ag;
    double h1 = sg * Pp.z - zs, h2 = sg * Sp.z - zs;
    double xc = (D * D + (h2 - h1) * (h2 + h1)) / (2.0 * D);
    double R = hypot(xc, h1);
    v3 uh = mk(dv.x / D, dv.y / D, 0.0);
    double sin0 = xc / R, cos0 = h1 / R;
    double sin1 = (xc - D) / R, cos1 = h2 / R;
    c.w_out = mk(cos0 * uh.x, cos0 * uh.y, sg * sin0);
    c.arrive = mk(cos1 * uh.x, cos1 * uh.y, sg * sin1);
    /* angle subtended at the centre between the radii to P and to S */
    double cr = xc * (h1 - h2) - h1 * D;     /* (-xc, h1) x (D - xc, h2) */
    double dt = -xc * (D - xc) + h1 * h2;
    double ang = atan2(fabs(cr), dt);
    c.L = R * ang;
    /* time: (atanh sin0 - atanh sin1) / |g| with sin0 - sin1 = D / R */
    double lc = log1p(ag * (h2 - h1) / (ag * h1));   /* ln(c_S / c_P) */
    double t;
    if (sin0 >= 0.0) t = log1p((D / R) / (1.0 + sin1)) + lc;
    else t = log1p((D / R) / (1.0 - sin0)) - lc;
    c.T = t / ag;
    c.path = make_path(P, Pp, c.w_out);
    return c;
}

/* Exposed for closed-form checks: eigenray P -> S. out = {L, T, w_out xyz, arrive xyz}. */
void orc_connection(const orc_params *P, const double p[3], const double s[3], double out[8])
{
    oconn c = connection(P, mk(p[0], p[1], p[2]), mk(s[0], s[1], s[2]));
    out[0] = c.L; out[1] = c.T;
    out[2] = c.w_out.x; out[3] = c.w_out.y; out[4] = c.w_out.z;
    out[5] = c.arrive.x; out[6] = c.arrive.y; out[7] = c.arrive.z;
}

/* Exposed: point, tangent and time after arc length s from (o, d). out = {x3, t3, time}. */
void orc_path_eval(const orc_params *P, const double o[3], const double d[3], double s, double out[7])
{
    opath p = make_path(P, mk(o[0], o[1], o[2]), mk(d[0], d[1], d[2]));
    v3 x = path_point(&p, s), t = path_tangent(&p, s);
    out[0] = x.x; out[1] = x.y; out[2] = x.z;
    out[3] = t.x; out[4] = t.y; out[5] = t.z;
    out[6] = path_time(P, &p, s);
}

/* ------------------------------------------------------------------------ */
/* Eigenrays through a layered profile. Snell's law keeps xi = cos(theta) / c */
/* fixed along a ray (theta the grazing angle), so crossing one layer between */
/* depths za and zb without turning, with s = |sin theta| = sqrt(1 - xi^2 c^2), */
/* the ray advances horizontally by X = integral of cot(theta) dz, travels arc */
/* length L = integral of dz / s and takes time T = integral of dz / (c s):     */
/*   X = (sa - sb) / (xi g)  = xi |dz| (ca + cb) / (sa + sb)                  */
/*   L = |asin sa - asin sb| / (xi |g|),  sin of that difference = xi g dz m,  */
/*       m = (ca + cb) / (sa cb + sb ca)                                      */
/*   T = |atanh sa - atanh sb| / |g| = |ln(1 + g dz (1 + m) / ((1 + sb) ca))| / |g| */
/* (each right-hand form is the left one rearranged without cancellation; the  */
/* straight-line limits g -> 0 and xi -> 0 follow). A turning point is where   */
/* s reaches 0. The return path from a vertex P to the sensor S is taken as    */
/* the eigenray with at most one turning point that arrives first: the direct */
/* ray (depth monotone between them), or one that turns above the higher of    */
/* the two depths or below the lower one.                                     */

typedef struct { double X, L, T; } orun;

/* c(zb) - c(za) as the sum of gradient times depth over the layers between
 * them: accurate relative to the difference itself, however close the two
 * speeds are (near a turning point 1 - xi c is such a difference). */
static double dspeed(const orc_params *P, double za, double zb)
{
    const int nl = layer_count(P);
    const double lo = fmin(za, zb), hi = fmax(za, zb);
    double sum = 0.0;
    for (int i = 0; i < nl; ++i) {
        const double a = i > 0 ? fmax(lo, P->knot_z[i]) : lo;
        const double b = i + 1 < nl ? fmin(hi, P->knot_z[i + 1]) : hi;
        if (b > a) sum += layer_g(P, i) * (b - a);
    }
    return zb >= za ? sum : -sum;
}

/* A ray family's invariant: xi = (1 - u) / c(zr), with zr the turning depth
 * (u = 0) or, for the direct family, the depth of the span's largest speed. */
typedef struct { double zr, u, cr, xi; } oref;

static oref ref_of(const orc_params *P, double zr, double u)
{
    oref R;
    R.zr = zr;
    R.u = u;
    R.cr = profile_c(P, zr);
    R.xi = (1.0 - u) / R.cr;
    return R;
}

/* |sin theta| at depth z: from 1 - xi c(z) = (c(zr) - c(z) + u c(z)) / c(zr) */
static double snell_sin(const orc_params *P, const oref *R, double z)
{
    const double a = (dspeed(P, z, R->zr) + R->u * profile_c(P, z)) / R->cr;
    return a <= 0.0 ? 0.0 : sqrt(a * (2.0 - a));
}

/* run of a ray of invariant R between depths za and zb of layer i */
static orun layer_run(const orc_params *P, const oref *R, int i, double za, double zb)
{
    orun r = {0.0, 0.0, 0.0};
    const double dz = zb - za, adz = fabs(dz);
    if (adz == 0.0) return r;
    const double g = layer_g(P, i), c0 = layer_c0(P, i), xi = R->xi;
    const double ca = c0 + g * za, cb = c0 + g * zb;
    const double sa = snell_sin(P, R, za), sb = snell_sin(P, R, zb);
    if (sa + sb == 0.0) {
        /* horizontal at both ends: in a constant layer the ray never leaves its
         * depth; otherwise the run is a rounding-level sliver at a turning point */
        if (g == 0.0) { r.X = r.L = r.T = HUGE_VAL; }
        else { r.L = adz; r.T = adz / ca; }
        return r;
    }
    r.X = xi * adz * (ca + cb) / (sa + sb);
    const double m = (ca + cb) / (sa * cb + sb * ca);
    const double y = fmin(1.0, xi * fabs(g) * adz * m);
    r.L = adz * m * (y > 0.0 ? asin(y) / y : 1.0);
    const double q = (1.0 + m) / ((1.0 + sb) * ca);
    r.T = g != 0.0 ? fabs(log1p(g * dz * q) / g) : adz * q;
    return r;
}

/* run between depths z0 <= z1, crossing every layer in between once */
static orun span_run(const orc_params *P, const oref *R, double z0, double z1)
{
    orun r = {0.0, 0.0, 0.0};
    const int nl = layer_count(P);
    int i = layer_of(P, z0);
    double za = z0;
    while (za < z1) {
        const double top = i + 1 < nl ? P->knot_z[i + 1] : HUGE_VAL;
        const double zb = top < z1 ? top : z1;
        const orun q = layer_run(P, R, i, za, zb);
        r.X += q.X; r.L += q.L; r.T += q.T;
        za = zb;
        ++i;
    }
    return r;
}

/* family 0: direct; 1: turning at depth zt above zhi; 2: turning at zt below zlo */
static orun eig_run(const orc_params *P, int fam, const oref *R, double zlo, double zhi)
{
    orun a = span_run(P, R, zlo, zhi);
    if (fam != 0) {
        const orun b = fam == 1 ? span_run(P, R, zhi, R->zr) : span_run(P, R, R->zr, zlo);
        a.X += 2.0 * b.X; a.L += 2.0 * b.L; a.T += 2.0 * b.T;
    }
    return a;
}

/* Turning depths of family 1 (above zhi) or 2 (below zlo) within H of the
 * span: the depths where c exceeds every speed met on the way there from the
 * span (cm = the largest speed on the span). At most one interval per layer;
 * returns their number, each as [nearer end, farther end] along the walk. */
static int turn_intervals(const orc_params *P, int fam, double zlo, double zhi, double cm, double H,
                          double iv[][2])
{
    const int nl = layer_count(P);
    int n = 0;
    double M = cm;
    if (fam == 1) {
        const double zend = zhi + H;
        int i = layer_of(P, zhi);
        double z = zhi;
        while (z < zend && i < nl) {
            const double top = i + 1 < nl ? P->knot_z[i + 1] : HUGE_VAL;
            const double zb = top < zend ? top : zend;
            const double g = layer_g(P, i), c0 = layer_c0(P, i);
            if (g > 0.0) {
                const double zs = (M - c0) / g;      /* c reaches the record here */
                const double a = zs > z ? zs : z;
                if (a < zb) { iv[n][0] = a; iv[n][1] = zb; ++n; }
                if (c0 + g * zb > M) M = c0 + g * zb;
            }
            z = zb;
            ++i;
        }
    } else {
        const double zend = zlo - H;
        int i = layer_of(P, zlo);
        if (i > 0 && zlo == P->knot_z[i]) --i;       /* going down from a knot: the layer below */
        double z = zlo;
        while (z > zend && i >= 0) {
            const double bot = i > 0 ? P->knot_z[i] : -HUGE_VAL;
            const double zb = bot > zend ? bot : zend;
            const double g = layer_g(P, i), c0 = layer_c0(P, i);
            if (g < 0.0) {
                const double zs = (M - c0) / g;
                const double a = zs < z ? zs : z;
                if (a > zb) { iv[n][0] = a; iv[n][1] = zb; ++n; }
                if (c0 + g * zb > M) M = c0 + g * zb;
            }
            z = zb;
            --i;
        }
    }
    return n;
}

#define EIG_SCAN 1024      /* scan cells over the turning-depth window (in v, below) */
#define EIG_MAXROOTS 256

typedef struct {
    int ok;            /* an eigenray was found */
    int fam, n_roots;
    double xi, zt;
    double L, T;
    v3 w_out, arrive;
    uint32_t flags;
} oeig;

typedef struct { int fam; double zr, u, T; } oroot;

static double eig_f(const orc_params *P, int fam, double zt, double zlo, double zhi, double D)
{
    const oref R = ref_of(P, zt, 0.0);
    return eig_run(P, fam, &R, zlo, zhi).X - D;
}

/* bisection of f between a (f <= 0 side or not, as classified) and b */
static double eig_bisect(const orc_params *P, int fam, double a, double b, double zlo, double zhi, double D)
{
    const int neg_a = eig_f(P, fam, a, zlo, zhi, D) <= 0.0;
    for (int it = 0; it < 200; ++it) {
        const double m = 0.5 * (a + b);
        if (m == a || m == b) break;
        if ((eig_f(P, fam, m, zlo, zhi, D) <= 0.0) == neg_a) a = m; else b = m;
    }
    return 0.5 * (a + b);
}

/* The first-arriving eigenray with at most one turning point from P to S.
 * The direct ray's invariant is found by bisection (its horizontal run grows
 * with xi up to xi = 1 / c_max of the span). Turning depths zt are searched
 * within H of the span on a grid uniform in v = sqrt(|zt - z_span| / H) (the
 * horizontal run of a turning ray grows like the square root of its rise),
 * EIG_SCAN cells plus the ends of the turning intervals, each sign change
 * refined by bisection. Flagged: a first arrival with another root of its
 * family closer than T->caustic in v (near a caustic, where a coarser search
 * could miss both; roots away from the first arrival do not change the
 * result), and a second arrival within T->tie_rel of the first in time. */
static oeig eigenray_layered(const orc_params *P, v3 Pp, v3 Sp, double H, const orc_tol *T)
{
    oeig e;
    memset(&e, 0, sizeof(e));
    const v3 dv = sub(Sp, Pp);
    const double D = hypot(dv.x, dv.y);
    const double zlo = fmin(Pp.z, Sp.z), zhi = fmax(Pp.z, Sp.z);
    double zm = profile_c(P, zlo) >= profile_c(P, zhi) ? zlo : zhi;     /* depth of the span's largest speed */
    for (int i = 0; i < P->n_knots; ++i)
        if (P->knot_z[i] > zlo && P->knot_z[i] < zhi && P->knot_c[i] > profile_c(P, zm)) zm = P->knot_z[i];
    const double cm = profile_c(P, zm);
    oroot roots[EIG_MAXROOTS];
    int nr = 0;
    /* direct family, xi = (1 - u) / cm: the run shrinks as u grows from 0 to 1 */
    if (zlo == zhi) {
        if (layer_g(P, layer_of(P, zlo)) == 0.0 && D > 0.0)
            roots[nr++] = (oroot){0, zm, 0.0, D / cm};            /* horizontal in a constant layer */
    } else {
        double a = 0.0, b = 1.0;
        const oref R0 = ref_of(P, zm, 0.0);
        if (D == 0.0) {
            a = b = 1.0;                                         /* vertical */
        } else if (span_run(P, &R0, zlo, zhi).X - D > 0.0) {
            for (int it = 0; it < 200; ++it) {
                const double m = 0.5 * (a + b);
                if (m == a || m == b) break;
                const oref R = ref_of(P, zm, m);
                if (span_run(P, &R, zlo, zhi).X - D > 0.0) a = m; else b = m;
            }
        } else {
            a = b = -1.0;                                        /* out of the direct family's reach */
        }
        if (a >= 0.0) {
            const double u = 0.5 * (a + b);
            const oref R = ref_of(P, zm, u);
            roots[nr++] = (oroot){0, zm, u, span_run(P, &R, zlo, zhi).T};
        }
    }
    /* turning families: scan the turning depth */
    for (int fam = 1; fam <= 2; ++fam) {
        double iv[ORC_MAXKNOTS + 1][2];
        const int ni = turn_intervals(P, fam, zlo, zhi, cm, H, iv);
        const double z0 = fam == 1 ? zhi : zlo, dir = fam == 1 ? 1.0 : -1.0;
        for (int q = 0; q < ni; ++q) {
            const double a = iv[q][0], b = iv[q][1];
            double zp = a;
            int negp = eig_f(P, fam, zp, zlo, zhi, D) <= 0.0;
            int j = (int)floor(sqrt(fabs(a - z0) / H) * EIG_SCAN) + 1;
            for (;; ++j) {
                const double v = (double)j / EIG_SCAN;
                double zq = z0 + dir * (H * (v * v));
                const int last = dir * (zq - b) >= 0.0;
                if (last) zq = b;
                if (dir * (zq - zp) <= 0.0) continue;       /* a grid point not past the interval start */
                const int negq = eig_f(P, fam, zq, zlo, zhi, D) <= 0.0;
                if (negq != negp) {
                    if (nr == EIG_MAXROOTS) {
                        e.flags |= F_CAUSTIC;       /* more roots than kept: not compared */
                    } else {
                        const double zt = eig_bisect(P, fam, zp, zq, zlo, zhi, D);
                        const oref R = ref_of(P, zt, 0.0);
                        roots[nr++] = (oroot){fam, zt, 0.0, eig_run(P, fam, &R, zlo, zhi).T};
                    }
                }
                if (last) break;
                zp = zq;
                negp = negq;
            }
        }
    }
    e.n_roots = nr;
    if (nr == 0) return e;
    int best = 0;
    for (int r = 1; r < nr; ++r)
        if (roots[r].T < roots[best].T) best = r;
    for (int r = 0; r < nr; ++r) {
        if (r == best) continue;
        if (roots[r].T <= roots[best].T * (1.0 + T->tie_rel)) e.flags |= F_CAUSTIC;
        if (roots[best].fam != 0 && roots[r].fam == roots[best].fam) {
            const double z0 = roots[best].fam == 1 ? zhi : zlo;
            if (fabs(sqrt(fabs(roots[r].zr - z0) / H) - sqrt(fabs(roots[best].zr - z0) / H)) < T->caustic)
                e.flags |= F_CAUSTIC;
        }
    }
    const oroot *B = &roots[best];
    const oref R = ref_of(P, B->zr, B->u);
    orun run = eig_run(P, B->fam, &R, zlo, zhi);
    if (B->fam == 0 && zlo == zhi) { run.L = D; run.T = D / cm; }
    e.ok = 1;
    e.fam = B->fam;
    e.xi = R.xi;
    e.zt = B->fam != 0 ? B->zr : 0.0;
    e.L = run.L;
    e.T = run.T;
    /* directions: horizontal part toward S, vertical sign by family and order */
    const v3 uh = D > 0.0 ? mk(dv.x / D, dv.y / D, 0.0) : mk(0.0, 0.0, 0.0);
    const double cp = R.xi * profile_c(P, Pp.z), cs = R.xi * profile_c(P, Sp.z);
    const double sp = snell_sin(P, &R, Pp.z), ss = snell_sin(P, &R, Sp.z);
    const double up = Sp.z > Pp.z ? 1.0 : (Sp.z < Pp.z ? -1.0 : 0.0);
    const double vp = B->fam == 0 ? up : (B->fam == 1 ? 1.0 : -1.0);
    const double vs = B->fam == 0 ? up : (B->fam == 1 ? -1.0 : 1.0);
    e.w_out = unit(mk(cp * uh.x, cp * uh.y, vp * sp));
    e.arrive = unit(mk(cs * uh.x, cs * uh.y, vs * ss));
    return e;
}

/* Occlusion of the layered eigenray leaving P along w for arc length L: the
 * path is walked one circle per layer and each piece is tested. */
static int blocked_layered(const oscene *S, const orc_params *P, v3 Pp, v3 w, double L, int64_t skip,
                           const orc_tol *T, uint32_t *flags)
{
    int layer = layer_of(P, Pp.z);
    if (layer > 0 && Pp.z == P->knot_z[layer] && w.z < 0.0) --layer;
    v3 o = Pp, d = w;
    double s0 = 0.0;
    for (int piece = 0; piece < 64; ++piece) {
        const double g = layer_g(P, layer), c0 = layer_c0(P, layer);
        opath path = make_path_gc(g, c0, o, d);
        int next;
        const double s_exit = layer_exit(P, layer, &path, g, c0, &next, flags);
        const double len = s_exit < L - s0 ? s_exit : L - s0;
        if (blocked_piece(S, &path, skip, s0, len, L, T, flags)) return 1;
        if (next < 0 || s0 + s_exit >= L) break;
        s0 += s_exit;
        o = path_point(&path, s_exit);
        d = unit(path_tangent(&path, s_exit));
        layer = next;
    }
    return 0;
}

/* Exposed for checks: the layered eigenray P -> S with turning depths within
 * H. out = {ok, family, roots, xi, zt, L, T, w xyz, arrive xyz, flags}. */
void orc_eigenray(const orc_params *P, const orc_tol *T, const double p[3], const double s[3], double H,
                  double out[14])
{
    const oeig e = eigenray_layered(P, mk(p[0], p[1], p[2]), mk(s[0], s[1], s[2]), H, T);
    out[0] = e.ok; out[1] = e.fam; out[2] = e.n_roots; out[3] = e.xi; out[4] = e.zt;
    out[5] = e.L; out[6] = e.T;
    out[7] = e.w_out.x; out[8] = e.w_out.y; out[9] = e.w_out.z;
    out[10] = e.arrive.x; out[11] = e.arrive.y; out[12] = e.arrive.z;
    out[13] = (double)e.flags;
}

/* ------------------------------------------------------------------------ */
/* The per-ray model.                                                        */

typedef struct {
    int32_t tri[ORC_MAXK], bin[ORC_MAXK], vis[ORC_MAXK], rxb[ORC_MAXK];
    double re[ORC_MAXK], im[ORC_MAXK], inc[ORC_MAXK];
    int32_t rbin[ORC_MAXK];                        /* retro-chain return of each vertex */
    double rre[ORC_MAXK], rim[ORC_MAXK], rinc[ORC_MAXK];
    uint32_t flags;
    int g_valid;
    double g_r, g_cos, g_rho;
    v3 g_n;
} oray;

static double upper_speed(const orc_params *P, const oscene *S, const orc_pose *Q)
{
    /* an upper bound of c(z) over the scene and the sensor, with 1 m margin */
    double z = S->zabs_max;
    if (fabs(Q->pos[2]) > z) z = fabs(Q->pos[2]);
    if (P->n_knots >= 2) {
        /* c is linear between knots: its largest value over [-z-1, z+1] is at an end or a knot */
        double c = profile_c(P, z + 1.0), c2 = profile_c(P, -z - 1.0);
        if (c2 > c) c = c2;
        for (int i = 0; i < P->n_knots; ++i)
            if (fabs(P->knot_z[i]) <= z + 1.0 && P->knot_c[i] > c) c = P->knot_c[i];
        return c;
    }
    return P->c0 + fabs(P->g) * (z + 1.0);
}

/* orthonormal basis (t1, t2) around the unit vector n (Duff et al., JCGT 2017) */
static void onb(v3 n, v3 *t1, v3 *t2)
{
    const double sg = n.z >= 0.0 ? 1.0 : -1.0;
    const double a = -1.0 / (sg + n.z), b = n.x * n.y * a;
    *t1 = mk(1.0 + sg * n.x * n.x * a, sg * b, -sg * n.x);
    *t2 = mk(b, sg + n.y * n.y * a, -n.y);
}

/* The drawn continuation (unit) after vertex k of ray `ray`; returns 0 when it
 * does not leave the lit side (np faces the incoming ray). */
static int draw_continuation(const orc_params *P, uint64_t ray, int k, v3 rh, v3 np, double kd, double ks,
                             double *cos_out, v3 *out)
{
    const uint64_t c = ((uint64_t)P->ping << 40) ^ (ray << 2) ^ (uint64_t)k;
    const uint64_t z = orc_splitmix64_nth(P->seed ^ 0xD1B54A32D192ED03ULL, c + 1);
    const double u1 = (double)(z >> 40) / 16777216.0, u2 = (double)((z >> 16) & 0xFFFFFFu) / 16777216.0;
    const double u3 = (double)(z & 0xFFFFu) / 65536.0;
    v3 axis;
    double ca;
    if (u3 < ks / (kd + ks)) {
        axis = rh;
        ca = pow(1.0 - u1, 1.0 / (P->phong_n + 1.0));
    } else {
        axis = np;
        ca = sqrt(1.0 - u1);
    }
    const double sa = sqrt(fmax(0.0, 1.0 - ca * ca)), ph = 2.0 * ORC_PI * u2;
    v3 t1, t2;
    onb(axis, &t1, &t2);
    *out = unit(add(scl(axis, ca), add(scl(t1, sa * cos(ph)), scl(t2, sa * sin(ph)))));
    *cos_out = dot(*out, np);
    return *cos_out > 0.0;
}

static double lobe_gauss(double d_az, double d_el, double dh, double dv)
{
    const double a = d_az / dh, e = d_el / dv;
    return exp(-2.0 * log(2.0) * (a * a + e * e));
}

/* beam = launch beam index (or -1: beam options unused); d_az, d_el = the
 * launch direction's offsets from that beam's centre */
static void trace_ray(const oscene *S, const orc_params *P, const orc_pose *Q, const orc_tol *T,
                      v3 o, v3 d, int32_t beam, double d_az, double d_el, uint64_t ray_id, oray *out)
{
    memset(out, 0, sizeof(*out));
    for (int k = 0; k < ORC_MAXK; ++k) { out->tri[k] = -1; out->bin[k] = -1; out->rxb[k] = beam; out->rbin[k] = -1; }
    const double dh = P->hfov / P->n_h, dv = P->vfov / P->n_v;
    const int pattern = beam >= 0 && (P->flags & ORC_BEAM_PATTERN);
    const int rx_bin = beam >= 0 && (P->flags & ORC_RX_BEAMS);
    const double w_tx = pattern ? lobe_gauss(d_az, d_el, dh, dv) : 1.0;
    const int K = P->max_bounces;
    const v3 Sp = mk(Q->pos[0], Q->pos[1], Q->pos[2]);
    const int layered = P->n_knots >= 2;
    const double c_ref = layered ? profile_c(P, Sp.z) : P->c0 + P->g * Sp.z;   /* time-to-range speed */
    const double c_hi = upper_speed(P, S, Q);
    const double dr = (P->r_max - P->r_min) / P->n_bins;
    double L_out = 0.0, T_out = 0.0, W = 1.0;
    int64_t prev = -1;
    for (int k = 0; k < K; ++k) {
        ohit h;
        double tau, s_len;
        v3 X, din;
        if (layered) {
            /* through the layers: one circle per layer, in order */
            const double T_lim = (K == 1) ? P->r_max / c_ref : 2.0 * P->r_max / c_ref - T_out;
            int layer = layer_of(P, o.z);
            /* a sensor exactly on a knot, looking down, starts in the layer below */
            if (layer > 0 && o.z == P->knot_z[layer] && d.z < 0.0) --layer;
            double t_acc = 0.0, s_acc = 0.0;
            v3 po = o, pd = d;
            h.tri = -1;
            for (int piece = 0; piece < 64; ++piece) {
                const double g = layer_g(P, layer), c0 = layer_c0(P, layer);
                opath path = make_path_gc(g, c0, po, pd);
                int next;
                const double s_exit = layer_exit(P, layer, &path, g, c0, &next, &out->flags);
                const double s_cap = c_hi * (T_lim - t_acc);
                const double s_end = s_exit < s_cap ? s_exit : s_cap;
                h = nearest_hit_from(S, &path, prev, piece == 0 ? EPS_SELF : 0.0, s_end, T);
                out->flags |= h.flags;
                if (h.tri >= 0) {
                    tau = t_acc + path_time_gc(g, c0, &path, h.s);
                    s_len = s_acc + h.s;
                    X = path_point(&path, h.s);
                    din = path_tangent(&path, h.s);
                    break;
                }
                if (next < 0 || s_exit >= s_cap) break;
                t_acc += path_time_gc(g, c0, &path, s_exit);
                s_acc += s_exit;
                po = path_point(&path, s_exit);
                pd = unit(path_tangent(&path, s_exit));
                layer = next;
            }
            if (h.tri < 0) break;
            if (fabs(tau - T_lim) <= T->lim_rel * T_lim) out->flags |= F_LIMIT;
            if (tau > T_lim) break;
        } else {
            opath path = make_path(P, o, d);
            double s_lim, T_lim = 0.0;
            if (P->g == 0.0) {
                s_lim = (K == 1) ? P->r_max : 2.0 * P->r_max - L_out;
            } else {
                T_lim = (K == 1) ? P->r_max / c_ref : 2.0 * P->r_max / c_ref - T_out;
                s_lim = c_hi * T_lim;
            }
            if (s_lim <= EPS_SELF) break;
            h = nearest_hit(S, &path, prev, s_lim, T);
            out->flags |= h.flags;
            if (h.tri < 0) break;
            tau = path_time(P, &path, h.s);
            if (P->g != 0.0) {
                if (fabs(tau - T_lim) <= T->lim_rel * T_lim) out->flags |= F_LIMIT;
                if (tau > T_lim) break;
            }
            X = path_point(&path, h.s);
            din = path_tangent(&path, h.s);
            s_len = h.s;
        }
        L_out += s_len;
        T_out += tau;
        int64_t f = h.tri;
        out->tri[k] = (int32_t)f;

        /* two-sided facet: n' faces the incoming ray */
        v3 nh = unit(tri_normal(S, f));
        double dn = dot(nh, din);
        v3 np = dn > 0.0 ? scl(nh, -1.0) : nh;
        double cos_i = -dot(np, din);
        if (cos_i < T->graze) out->flags |= F_GRAZE;
        v3 rh = sub(din, scl(np, 2.0 * dot(np, din)));      /* mirror direction */

        /* material: pressure-release facets have rho = 1, no diffuse part, a
         * unit specular part, phase 0 and reflection sign -1 */
        int pr = S->mat[f] == 1;
        double rho = pr ? 1.0 : S->rho[f];
        double kd = pr ? 0.0 : P->k_d;
        double ks = pr ? 1.0 : P->k_s;
        double phi = pr ? 0.0 : S->phi[f];
        double sgn = pr ? -1.0 : 1.0;

        /* return path */
        double L_back, T_back;
        v3 w;
        int vis = 1;
        double w_rx = w_tx;                 /* bounce 1: arrival along the launch ray */
        int32_t rxb = beam;
        if (k == 0) {
            L_back = L_out; T_back = T_out; w = scl(din, -1.0);
        } else {
            v3 arrive;
            uint32_t fl = 0;
            if (layered) {
                /* the first-arriving eigenray, turning within 2 r_max of the span */
                const oeig e = eigenray_layered(P, X, Sp, 2.0 * P->r_max, T);
                fl |= e.flags;
                if (!e.ok) {
                    vis = 0;            /* no eigenray: the vertex lies in a shadow zone */
                    L_back = T_back = 0.0;
                    w = arrive = mk(0.0, 0.0, 0.0);
                } else {
                    L_back = e.L; T_back = e.T; w = e.w_out; arrive = e.arrive;
                    if (blocked_layered(S, P, X, w, e.L, f, T, &fl)) vis = 0;
                }
            } else {
                oconn c = connection(P, X, Sp);
                L_back = c.L; T_back = c.T; w = c.w_out; arrive = c.arrive;
                if (blocked(S, &c.path, f, c.L, T, &fl)) vis = 0;
            }
            out->flags |= fl;
            /* arrival direction must lie in the field of view */
            v3 a = world_to_sensor(Q, scl(arrive, -1.0));
            double az = atan2(a.y, a.x), el = atan2(a.z, hypot(a.x, a.y));
            double mh = 0.5 * P->hfov - fabs(az), mv = 0.5 * P->vfov - fabs(el);
            if (fabs(mh) <= T->fov || fabs(mv) <= T->fov) out->flags |= F_FOV;
            if (mh < 0.0 || mv < 0.0) vis = 0;
            if (beam >= 0 && vis && (pattern || rx_bin)) {
                const int nh = P->n_h;
                int h = beam % nh, v = beam / nh;
                if (rx_bin) {
                    /* the receive cell holding the arrival direction */
                    const double xa = (az + 0.5 * P->hfov) / dh, xe = (el + 0.5 * P->vfov) / dv;
                    h = (int)floor(xa);
                    v = (int)floor(xe);
                    if (h > P->n_h - 1) h = P->n_h - 1;
                    if (v > P->n_v - 1) v = P->n_v - 1;
                    if (h < 0) h = 0;
                    if (v < 0) v = 0;
                    /* an arrival within the FOV margin of a cell edge is ambiguous */
                    if (fabs(xa - floor(xa + 0.5)) * dh <= T->fov || fabs(xe - floor(xe + 0.5)) * dv <= T->fov)
                        out->flags |= F_FOV;
                    rxb = v * nh + h;
                }
                const double c_az = -0.5 * P->hfov + (h + 0.5) * dh, c_el = -0.5 * P->vfov + (v + 0.5) * dv;
                w_rx = pattern ? lobe_gauss(az - c_az, el - c_el, dh, dv) : 1.0;
            }
        }
        out->rxb[k] = rxb;
        out->vis[k] = vis;
        if (vis) {
            double cos_o = dot(np, w);
            if (k > 0 && fabs(cos_o) < T->graze) out->flags |= F_DEPART;
            if (cos_o > 0.0) {
                double Tt = T_out + T_back;
                double reff = c_ref * Tt / 2.0;
                double x = (reff - P->r_min) / dr;
                double fb = floor(x);
                double fr = x - fb;
                if (x > -1.0 && x < P->n_bins + 1.0 && (fr < T->bin_frac || fr > 1.0 - T->bin_frac))
                    out->flags |= F_BIN;
                if (fb >= 0.0 && fb < P->n_bins) {
                    int bin = (int)fb;
                    double lobe = dot(rh, w);
                    if (lobe < 0.0) lobe = 0.0;
                    double fsc = rho * (kd * cos_i * cos_o + ks * pow(lobe, P->phong_n));
                    double amp = W * sgn * sqrt(fsc) * pow(10.0, -P->alpha_db * (L_out + L_back) / 20.0) /
                                 (L_out * L_back * P->n_r);
                    if (pattern) amp *= w_tx * w_rx;
                    double cyc = P->f0 * Tt;
                    double ph = 2.0 * ORC_PI * (cyc - floor(cyc)) + phi;
                    out->bin[k] = bin;
                    out->re[k] = amp * cos(ph);
                    out->im[k] = amp * sin(ph);
                    out->inc[k] = amp * amp;
                    if (k == 0) {
                        out->g_valid = 1;
                        out->g_r = reff;
                        out->g_cos = cos_i;
                        out->g_rho = rho;
                        out->g_n = np;
                    }
                }
            }
        }
        /* retro-chain return: back into the reversed incident direction and
         * along the outgoing chain reversed */
        if (k > 0 && (P->flags & ORC_RETRO_CHAIN)) {
            double lobe = -dot(rh, din);
            if (lobe < 0.0) lobe = 0.0;
            const double fsc = rho * (kd * cos_i * cos_i + ks * pow(lobe, P->phong_n));
            const double Tt = 2.0 * T_out;
            const double reff = c_ref * Tt / 2.0;
            const double x = (reff - P->r_min) / dr, fb = floor(x), fr = x - fb;
            if (x > -1.0 && x < P->n_bins + 1.0 && (fr < T->bin_frac || fr > 1.0 - T->bin_frac))
                out->flags |= F_BIN;
            if (fb >= 0.0 && fb < P->n_bins) {
                double amp = W * W * sgn * sqrt(fsc) * pow(10.0, -P->alpha_db * 2.0 * L_out / 20.0) /
                             (L_out * L_out * P->n_r);
                if (pattern) amp *= w_tx * w_tx;
                const double cyc = P->f0 * Tt;
                const double ph = 2.0 * ORC_PI * (cyc - floor(cyc)) + phi;
                out->rbin[k] = (int)fb;
                out->rre[k] = amp * cos(ph);
                out->rim[k] = amp * sin(ph);
                out->rinc[k] = amp * amp;
            }
        }
        /* continuation along the mirror direction, or drawn from the lobes */
        if (k + 1 >= K) break;
        if ((P->flags & ORC_DIFFUSE_BOUNCE) && !pr) {
            W *= sqrt(rho * (kd + ks)) * sgn;
            if (W == 0.0) break;
            double cd;
            v3 nd;
            const int lit = draw_continuation(P, ray_id, k, rh, np, kd, ks, &cd, &nd);
            if (fabs(cd) < T->graze) out->flags |= F_DEPART;
            if (!lit) break;
            rh = nd;
        } else {
            W *= sqrt(rho * ks) * sgn;
        }
        if (W == 0.0) break;
        double dS = len(sub(X, Sp));
        double lb, bound;
        if (P->g == 0.0 && !layered) { lb = (L_out + dS) / 2.0; bound = P->r_max; }
        else { lb = c_ref * (T_out + dS / c_hi) / 2.0; bound = P->r_max; }
        if (fabs(lb - bound) <= T->lim_rel * bound) out->flags |= F_STOP;
        if (lb >= bound) break;
        o = X; d = rh; prev = f;
    }
}

/* ------------------------------------------------------------------------ */
/* Beams: all rays of each listed beam, their records, and the beam's range   */
/* column. Every ray of a bundle is weighted 1/N_r and contributes to its    */
/* launch beam (the complex sum over the beam's bundle of rays).            */

int orc_trace_beams(void *hs, const orc_params *P, const orc_pose *Q, const orc_tol *T,
                    const int32_t *beams, int64_t n_beams,
                    double *col,        /* [n_beams][n_bins][2], flagged rays excluded */
                    double *col_all,    /* [n_beams][n_bins][2], every ray, or NULL */
                    double *incoh,      /* [n_beams][2][n_bins] (bounce 1, bounces >= 2), or NULL */
                    double *gbuf,       /* [n_beams][8], or NULL */
                    int32_t *rec_tri, int32_t *rec_bin, int32_t *rec_vis,  /* [n_beams*n_r][K] */
                    double *rec_amp,    /* [n_beams*n_r][K][2] */
                    uint32_t *ray_flags,/* [n_beams*n_r] */
                    int32_t *rec_rxb,   /* [n_beams*n_r][K] receive beam of each contribution, or NULL */
                    int32_t *rec_rbin,  /* [n_beams*n_r][K] retro-chain bin of each vertex, or NULL */
                    double *rec_ramp,   /* [n_beams*n_r][K][2] retro-chain contribution, or NULL */
                    int n_threads)
{
    const oscene *S = (const oscene *)hs;
    if (P->max_bounces < 1 || P->max_bounces > ORC_MAXK) return -1;
    const int K = P->max_bounces, NB = P->n_bins, NR = P->n_r;
    if ((P->flags & (ORC_BEAM_PATTERN | ORC_RX_BEAMS)) && P->grid_mode != 0)
        return -3;                                           /* beam options: cell-centred beams only */
    if (P->n_knots != 0) {
        /* a layered profile: 2..8 knots with increasing depth and positive speed */
        if (P->n_knots < 2 || P->n_knots > ORC_MAXKNOTS) return -5;
        for (int i = 0; i < P->n_knots; ++i) {
            if (!(P->knot_c[i] > 0.0)) return -5;
            if (i > 0 && !(P->knot_z[i] > P->knot_z[i - 1])) return -5;
        }
    }
    const int rx = (P->flags & ORC_RX_BEAMS) != 0;
    if ((P->flags & ORC_RETRO_CHAIN) && rx && (!rec_rbin || !rec_ramp)) return -4;
    /* receive binning moves contributions between beams: the columns need
     * every beam, in order; for a subset of beams only the records are
     * filled (columns zero) */
    int rx_all = rx && n_beams == (int64_t)P->n_h * P->n_v;
    for (int64_t q = 0; rx_all && q < n_beams; ++q)
        if (beams[q] != q) rx_all = 0;
    const double dh = P->hfov / P->n_h, dv = P->vfov / P->n_v;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < n_beams; ++q) {
        int b = beams[q];
        double *cc = col + (size_t)q * NB * 2;
        double *ca = col_all ? col_all + (size_t)q * NB * 2 : NULL;
        double *ic = incoh ? incoh + (size_t)q * 2 * NB : NULL;
        memset(cc, 0, sizeof(double) * NB * 2);
        if (ca) memset(ca, 0, sizeof(double) * NB * 2);
        if (ic) memset(ic, 0, sizeof(double) * NB * 2);
        double gs[8] = {0};
        int gcount = 0;
        for (int j = 0; j < NR; ++j) {
            double od[6];
            orc_ray(P, Q, b, j, od);
            double d_az = 0.0, d_el = 0.0;
            if (P->flags & (ORC_BEAM_PATTERN | ORC_RX_BEAMS)) {
                double az, el;
                ray_angles(P, b, j, &az, &el);
                const int nh = beams_h(P);
                d_az = az - (-0.5 * P->hfov + (b % nh + 0.5) * dh);
                d_el = el - (-0.5 * P->vfov + (b / nh + 0.5) * dv);
            }
            oray r;
            trace_ray(S, P, Q, T, mk(od[0], od[1], od[2]), mk(od[3], od[4], od[5]),
                      (P->flags & (ORC_BEAM_PATTERN | ORC_RX_BEAMS)) ? b : -1, d_az,
                      d_el, (uint64_t)b * NR + j, &r);
            size_t ri = (size_t)q * NR + j;
            ray_flags[ri] = r.flags;
            for (int k = 0; k < K; ++k) {
                rec_tri[ri * K + k] = r.tri[k];
                rec_bin[ri * K + k] = r.bin[k];
                rec_vis[ri * K + k] = r.vis[k];
                rec_amp[(ri * K + k) * 2] = r.re[k];
                rec_amp[(ri * K + k) * 2 + 1] = r.im[k];
                if (rec_rxb) rec_rxb[ri * K + k] = r.rxb[k] >= 0 ? r.rxb[k] : b;
                if (rx) r.inc[k] = r.re[k] * r.re[k] + r.im[k] * r.im[k];
                if (rec_rbin) rec_rbin[ri * K + k] = r.rbin[k];
                if (rec_ramp) { rec_ramp[(ri * K + k) * 2] = r.rre[k]; rec_ramp[(ri * K + k) * 2 + 1] = r.rim[k]; }
                if (rx) continue;
                if (r.bin[k] >= 0) {
                    if (ca) { ca[2 * r.bin[k]] += r.re[k]; ca[2 * r.bin[k] + 1] += r.im[k]; }
                    if (r.flags == 0) {
                        cc[2 * r.bin[k]] += r.re[k];
                        cc[2 * r.bin[k] + 1] += r.im[k];
                        if (ic) ic[(k == 0 ? 0 : NB) + r.bin[k]] += r.inc[k];
                    }
                }
                if (r.rbin[k] >= 0) {
                    if (ca) { ca[2 * r.rbin[k]] += r.rre[k]; ca[2 * r.rbin[k] + 1] += r.rim[k]; }
                    if (r.flags == 0) {
                        cc[2 * r.rbin[k]] += r.rre[k];
                        cc[2 * r.rbin[k] + 1] += r.rim[k];
                        if (ic) ic[NB + r.rbin[k]] += r.rinc[k];
                    }
                }
            }
            if (r.flags == 0 && r.g_valid) {
                gs[0] += r.g_r / P->r_max;
                gs[1] += r.g_cos;
                gs[2] += r.g_rho;
                gs[3] += r.g_n.x; gs[4] += r.g_n.y; gs[5] += r.g_n.z;
                ++gcount;
            }
        }
        if (gbuf) {
            double *g = gbuf + (size_t)q * 8;
            for (int t = 0; t < 8; ++t) g[t] = 0.0;
            if (gcount > 0) for (int t = 0; t < 6; ++t) g[t] = gs[t] / gcount;
            g[6] = (double)gcount / NR;
            /* the beam axis in the world frame: its vertical component */
            const int nh = beams_h(P);
            const double off = P->grid_mode == 1 ? 0.0 : 0.5;
            const double az = -0.5 * P->hfov + (b % nh + off) * dh, el = -0.5 * P->vfov + (b / nh + off) * dv;
            g[7] = sensor_to_world(Q, dir_from_angles(az, el)).z;
        }
    }
    if (rx) {
        /* receive binning: columns from the records, in ray order */
        for (int64_t q = 0; q < n_beams; ++q) {
            memset(col + (size_t)q * NB * 2, 0, sizeof(double) * NB * 2);
            if (col_all) memset(col_all + (size_t)q * NB * 2, 0, sizeof(double) * NB * 2);
            if (incoh) memset(incoh + (size_t)q * 2 * NB, 0, sizeof(double) * NB * 2);
        }
        if (!rx_all) return 0;
        for (size_t ri = 0; ri < (size_t)n_beams * NR; ++ri) {
            for (int k = 0; k < K; ++k) {
                const size_t e = ri * K + k;
                const int bin = rec_bin[e];
                if (bin < 0) continue;
                /* the receive beam (records carry it when asked for; else recompute below) */
                int32_t tb = rec_rxb ? rec_rxb[e] : -1;
                if (tb < 0) return -4;
                const double re = rec_amp[2 * e], im = rec_amp[2 * e + 1];
                if (col_all) { col_all[((size_t)tb * NB + bin) * 2] += re; col_all[((size_t)tb * NB + bin) * 2 + 1] += im; }
                if (ray_flags[ri] == 0) {
                    col[((size_t)tb * NB + bin) * 2] += re;
                    col[((size_t)tb * NB + bin) * 2 + 1] += im;
                    if (incoh) incoh[(size_t)tb * 2 * NB + (k == 0 ? 0 : NB) + bin] += re * re + im * im;
                }
            }
            /* retro-chain returns arrive along the launch ray: the launch beam */
            for (int k = 0; rec_rbin && k < K; ++k) {
                const size_t e = ri * K + k;
                const int bin = rec_rbin[e];
                if (bin < 0) continue;
                const size_t tb = ri / NR;
                const double re = rec_ramp[2 * e], im = rec_ramp[2 * e + 1];
                if (col_all) { col_all[(tb * NB + bin) * 2] += re; col_all[(tb * NB + bin) * 2 + 1] += im; }
                if (ray_flags[ri] == 0) {
                    col[(tb * NB + bin) * 2] += re;
                    col[(tb * NB + bin) * 2 + 1] += im;
                    if (incoh) incoh[tb * 2 * NB + NB + bin] += re * re + im * im;
                }
            }
        }
    }
    return 0;
}

/* The drawn continuation of ray `ray` after vertex k (distribution checks):
 * out = direction xyz, cos with np, lit flag. */
void orc_draw_continuation(const orc_params *P, uint64_t ray, int32_t k, const double rh[3], const double np[3],
                           double kd, double ks, double out[5])
{
    double c;
    v3 d;
    const int lit = draw_continuation(P, ray, k, mk(rh[0], rh[1], rh[2]), mk(np[0], np[1], np[2]), kd, ks, &c, &d);
    out[0] = d.x; out[1] = d.y; out[2] = d.z; out[3] = c; out[4] = lit;
}

/* A single ray from an arbitrary origin and direction (closed-form checks). */
int orc_trace_one(void *hs, const orc_params *P, const orc_pose *Q, const orc_tol *T,
                  const double o[3], const double d[3],
                  int32_t *tri, int32_t *bin, int32_t *vis, double *amp, uint32_t *flags,
                  int32_t *rbin, double *ramp)      /* retro-chain returns, or NULL */
{
    const oscene *S = (const oscene *)hs;
    if (P->max_bounces < 1 || P->max_bounces > ORC_MAXK) return -1;
    oray r;
    trace_ray(S, P, Q, T, mk(o[0], o[1], o[2]), unit(mk(d[0], d[1], d[2])), -1, 0.0, 0.0, 0, &r);
    for (int k = 0; k < P->max_bounces; ++k) {
        tri[k] = r.tri[k]; bin[k] = r.bin[k]; vis[k] = r.vis[k];
        amp[2 * k] = r.re[k]; amp[2 * k + 1] = r.im[k];
        if (rbin) rbin[k] = r.rbin[k];
        if (ramp) { ramp[2 * k] = r.rre[k]; ramp[2 * k + 1] = r.rim[k]; }
    }
    *flags = r.flags;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Detection: cell-averaging CFAR (Finn and Johnson 1968) on |E|^2 + N0 per    */
/* beam, a local-peak test, at most `max_per_beam` strongest cells per beam, */
/* and points at the beam centre along a straight line at the bin-centre     */
/* range. Flags mark decisions within a relative margin of their threshold.  */

typedef struct {
    int32_t train, guard, max_per_beam, pad;
    double pfa, noise_floor;
} orc_cfar;

int orc_detect(const float *vol, const orc_params *P, const orc_pose *Q, const orc_cfar *C,
               const int32_t *beams, int64_t n_beams,
               int32_t *out_bin,      /* [n_beams][max_per_beam], -1 padded, in range order */
               double *out_pts,       /* [n_beams][max_per_beam][4]: x, y, z, dB */
               int32_t *out_count,    /* [n_beams] */
               uint8_t *flag_bins,    /* [n_beams][n_bins]: 1 = decision near its threshold */
               int32_t *beam_flag,    /* [n_beams]: 1 = top-k choice ambiguous */
               double rel_thr, double rel_peak)
{
    const int NB = P->n_bins, M = C->max_per_beam;
    const double dr = (P->r_max - P->r_min) / NB;
    double *Pw = (double *)malloc(sizeof(double) * NB);
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * NB);
    for (int64_t q = 0; q < n_beams; ++q) {
        int b = beams[q];
        const float *col = vol + (size_t)b * NB * 2;
        for (int r = 0; r < NB; ++r) {
            double re = col[2 * r], im = col[2 * r + 1];
            Pw[r] = re * re + im * im + C->noise_floor;
        }
        uint8_t *fb = flag_bins + (size_t)q * NB;
        int nc = 0;
        for (int r = 0; r < NB; ++r) {
            fb[r] = 0;
            double sum = 0.0;
            int N = 0;
            for (int t = r - C->guard - C->train; t <= r + C->guard + C->train; ++t) {
                if (t < 0 || t >= NB) continue;
                if (t >= r - C->guard && t <= r + C->guard) continue;
                sum += Pw[t];
                ++N;
            }
            if (N == 0) continue;
            double alpha = N * (pow(C->pfa, -1.0 / N) - 1.0);
            double thr = alpha * sum / N;
            int det = Pw[r] > thr;
            if (fabs(Pw[r] - thr) <= rel_thr * thr) fb[r] = 1;
            if (r > 0) {
                if (!(Pw[r] > Pw[r - 1])) det = 0;
                if (fabs(Pw[r] - Pw[r - 1]) <= rel_peak * Pw[r]) fb[r] = 1;
            }
            if (r + 1 < NB) {
                if (!(Pw[r] >= Pw[r + 1])) det = 0;
                if (fabs(Pw[r] - Pw[r + 1]) <= rel_peak * Pw[r]) fb[r] = 1;
            }
            if (det) cand[nc++] = r;
        }
        /* keep the M strongest: power descending, then lower range */
        for (int a = 1; a < nc; ++a) {
            int x = cand[a], t = a - 1;
            while (t >= 0 && (Pw[cand[t]] < Pw[x] || (Pw[cand[t]] == Pw[x] && cand[t] > x))) {
                cand[t + 1] = cand[t];
                --t;
            }
            cand[t + 1] = x;
        }
        beam_flag[q] = 0;
        if (nc > M && fabs(Pw[cand[M - 1]] - Pw[cand[M]]) <= rel_peak * Pw[cand[M - 1]]) beam_flag[q] = 1;
        int kept = nc < M ? nc : M;
        /* output in range order */
        for (int a = 1; a < kept; ++a) {
            int x = cand[a], t = a - 1;
            while (t >= 0 && cand[t] > x) { cand[t + 1] = cand[t]; --t; }
            cand[t + 1] = x;
        }
        int nh = beams_h(P);
        int h = b % nh, v = b / nh;
        double az, el;
        if (P->grid_mode == 1) {
            az = -0.5 * P->hfov + h * (P->hfov / P->n_h);
            el = -0.5 * P->vfov + v * (P->vfov / P->n_v);
        } else {
            az = -0.5 * P->hfov + (h + 0.5) * (P->hfov / P->n_h);
            el = -0.5 * P->vfov + (v + 0.5) * (P->vfov / P->n_v);
        }
        v3 dw = sensor_to_world(Q, dir_from_angles(az, el));
        out_count[q] = kept;
        for (int a = 0; a < M; ++a) {
            out_bin[q * M + a] = a < kept ? cand[a] : -1;
            double *pt = out_pts + ((size_t)q * M + a) * 4;
            if (a < kept) {
                double rr = P->r_min + (cand[a] + 0.5) * dr;
                pt[0] = Q->pos[0] + dw.x * rr;
                pt[1] = Q->pos[1] + dw.y * rr;
                pt[2] = Q->pos[2] + dw.z * rr;
                pt[3] = 10.0 * log10(Pw[cand[a]]);
            } else {
                pt[0] = pt[1] = pt[2] = pt[3] = 0.0;
            }
        }
    }
    free(Pw);
    free(cand);
    return 0;
}
