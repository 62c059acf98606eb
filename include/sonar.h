/*
 * sonar.h -- C-ABI of the MI355X volumetric sonar echo-synthesis library
 * (libsonar.so, hand-written HIP for gfx950).
 *
 * The method (arXiv 2606.06130, "Towards Realistic 3D Sonar Simulation"):
 *   - Sec. II-A: the sensor is volumetric; its aperture is discretised in
 *     azimuth and elevation and each ping yields an azimuth x elevation x
 *     range distribution of backscatter. Rays are cast in parallel through
 *     the scene and bend by Snell's law in a sound-speed field.
 *   - Sec. II-B: every intersection scatters according to its incidence angle
 *     and material coefficients; a bounded, tunable number of secondary
 *     reflections; complex returns carry phase from the propagation delay and
 *     are attenuated; beams and cells are formed by coherent summation within
 *     each ray bundle.
 *   - Sec. III, Eq. (1)-(3): the sampling grid N_range, N_H, N_V from the
 *     fields of view, range limits and resolutions; the LiDAR firing grid has
 *     (N_V + 1) x (N_H + 1) emitters.
 *
 * Conventions shared by every entry point:
 *   - World frame: metres, z up. Sensor frame: x forward, y left, z up.
 *     Azimuth is measured from +x toward +y, elevation toward +z. Beam index
 *     b = v * beams_per_row + h, with h and v increasing with azimuth and
 *     elevation.
 *   - Volumes are complex64 [beams_v][beams_h][n_range], interleaved FP32
 *     (re, im), elevation-major: layout-compatible with torch.complex64.
 *   - Ownership: the caller owns every buffer passed in; the library owns only
 *     the scene it builds. Inputs of sonar_build_scene may be freed when it
 *     returns.
 *   - Streams: a sonar_stream is a hipStream_t (NULL = the null stream).
 *     Every call is stream-ordered and asynchronous except sonar_build_scene
 *     and sonar_device_status, which synchronise.
 *   - Errors: host-side validation runs before any launch; a failing call
 *     returns a negative status, launches nothing and leaves a message for
 *     sonar_last_error() (per thread). Nothing aborts and no C++ exception
 *     crosses this boundary. sonar_ping, sonar_ping_batch and sonar_detect
 *     allocate nothing.
 */
#ifndef SONAR_H
#define SONAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SONAR_OK = 0,
    SONAR_W_TRUNCATED = 1,      /* more detections than `capacity`; the count holds the total */
    SONAR_E_INVALID = -1,       /* an argument failed validation */
    SONAR_E_NOMEM = -2,         /* device allocation failed (build only) */
    SONAR_E_DEVICE = -3,        /* a HIP call failed */
    SONAR_E_STACK = -4,         /* traversal stack too shallow for the scene's hierarchy */
    SONAR_E_UNSUPPORTED = -5    /* a valid request outside what the library implements */
} sonar_status;

/* Opaque, library-owned, immutable after build. Usable from several streams
 * at once. */
typedef struct sonar_scene sonar_scene;

/* Triangle mesh with per-facet material metadata (Sec. II-B: reflection and
 * scattering coefficients per material; the engine provides geometry and
 * material data, the acoustic layer the rest).
 *   vertices     float32 [n_vertices][3], metres
 *   indices      int32 [n_triangles][3], each in [0, n_vertices)
 *   reflectivity float32 [n_triangles], intensity coefficient rho >= 0
 *   phase        float32 [n_triangles], per-facet phase (rad)
 *   material     uint8 [n_triangles]: 0 rough facet, 1 pressure-release
 *                surface (rho 1, no diffuse part, unit specular part,
 *                phase 0, reflection sign -1)
 *   on_device    0: host pointers, 1: device pointers
 *   leaf_size    most triangles per hierarchy leaf, 1..8 (0 = 3) */
typedef struct {
    const float *vertices;
    const int32_t *indices;
    const float *reflectivity;
    const float *phase;
    const uint8_t *material;
    int64_t n_vertices;
    int64_t n_triangles;
    int32_t on_device;
    int32_t leaf_size;
} sonar_mesh;

/* Sensor pose: position (metres) and sensor->world rotation, row-major, whose
 * columns are the sensor's x, y, z axes in world coordinates. `ping` is the
 * ping counter that keys the jitter sequence. */
typedef struct {
    double position[3];
    double rot[9];
    uint32_t ping;
    uint32_t pad;
} sonar_pose;

/* Sensor, medium and scattering parameters.
 *   hfov, vfov        fields of view (rad), Sec. III
 *   n_h, n_v          angular samples N_H, N_V (Eq. 2-3)
 *   rays_per_beam     rays per beam: a power of two in [1, 64]
 *   grid_mode         0: N_H x N_V cell-centred beams, rays stratified inside
 *                     each cell; 1: LiDAR firing grid of (N_V+1) x (N_H+1)
 *                     emitters at -FOV/2 + i * FOV/N (rays_per_beam must be 1)
 *   jitter            1: one uniform sample per stratum, 0: stratum centres
 *   n_range           range bins N_range (Eq. 1), 1..4096
 *   r_min, r_max      range limits (m); bin = floor((r - r_min) / dr),
 *                     dr = (r_max - r_min) / n_range
 *   freq_hz           centre frequency f0 (phase 2 pi f0 T)
 *   c0, c_grad        sound speed c(z) = c0 + c_grad * z (m/s)
 *   abs_db_per_m      absorption per metre of total (out + back) path
 *   max_bounces       path depth K, 1..4 (Sec. II-B: tunable)
 *   k_d, k_s, phong_n diffuse weight, specular weight, specular exponent
 *   seed              jitter seed (SplitMix64)
 *   flags             beam forming options (Sec. II-B: the contribution
 *                     depends on the transmit-receive beam pattern), 0 or:
 *     SONAR_FLAG_BEAM_PATTERN  weight every contribution by the one-way
 *                     amplitude pattern of the transmit beam at the launch
 *                     direction times that of the receive beam at the
 *                     arrival direction; a beam's pattern is the Gaussian
 *                     main lobe exp(-2 ln2 ((d_az/dth_h)^2 + (d_el/dth_v)^2))
 *                     in the angular offsets from its centre (one-way power
 *                     3 dB down half a cell off axis)
 *     SONAR_FLAG_RX_BEAMS  a return of bounce >= 2 goes to the receive beam
 *                     whose cell holds its arrival direction instead of the
 *                     launch beam (bounce-1 returns arrive along the reversed
 *                     launch ray); with max_bounces > 1 it needs the
 *                     workspace of sonar_ping_rx or sonar_ping_detect (in
 *                     batches: sonar_batch_prepare_rx)
 *                     Both options need cell-centred beams (grid_mode 0).
 *     SONAR_FLAG_DIFFUSE_BOUNCE  stochastic scattering (Sec. II-B: speckle,
 *                     reverberation): the continuation after a rough facet is
 *                     drawn from its lobes instead of the mirror direction,
 *                     the Phong lobe around the mirror with probability
 *                     k_s / (k_d + k_s) (cos a = (1 - u1)^(1 / (phong_n + 1)))
 *                     else the cosine lobe around the facet normal facing the
 *                     ray (cos a = sqrt(1 - u1)), azimuth 2 pi u2; the uniforms
 *                     come from SplitMix64 output c + 1 of (seed xor
 *                     0xD1B54A32D192ED03), c = (ping << 40) xor (ray << 2) xor
 *                     k (u1 = z >> 40, u2 = (z >> 16) mod 2^24 over 2^24,
 *                     u3 = z mod 2^16 over 2^16 chooses the lobe); the path
 *                     weight takes sqrt(rho (k_d + k_s)); a direction into the
 *                     facet ends the ray. Pressure-release facets stay mirrors.
 *     SONAR_FLAG_RETRO_CHAIN  retro-chain returns (Sec. II-B: secondary
 *                     reflections): every vertex after the first also
 *                     scatters back into its reversed incident direction and
 *                     the echo retraces the outgoing chain (the same path, so
 *                     no visibility test): time 2 T_out, spreading
 *                     1 / L_out^2, absorption over 2 L_out, the chain's path
 *                     weight squared, departure cosine = incidence cosine and
 *                     the Phong lobe toward the reversed incident direction;
 *                     it arrives along the launch ray (launch beam, transmit
 *                     pattern squared) and counts as a later bounce in the
 *                     incoherent channel. No effect with max_bounces 1;
 *                     rejected for n_range above 3328 (3 bounces) or 3584
 *                     (4 bounces); the pings of a batch take it all or none. */
#define SONAR_FLAG_BEAM_PATTERN 1u
#define SONAR_FLAG_RX_BEAMS 2u
#define SONAR_FLAG_DIFFUSE_BOUNCE 4u
#define SONAR_FLAG_RETRO_CHAIN 8u
typedef struct {
    double hfov, vfov;
    int32_t n_h, n_v, rays_per_beam, grid_mode, jitter, n_range;
    double r_min, r_max, freq_hz, c0, c_grad, abs_db_per_m;
    int32_t max_bounces, pad0;
    double k_d, k_s, phong_n;
    uint64_t seed;
    uint32_t flags, pad1;
} sonar_params;

/* CFAR detection settings (cell averaging): `train` training and `guard`
 * guard cells per side, probability of false alarm `pfa`, `noise_floor` added
 * to |E|^2, at most `max_per_beam` points per beam (1..16). */
typedef struct {
    int32_t train, guard, max_per_beam, pad;
    double pfa, noise_floor;
} sonar_cfar;

typedef struct { float x, y, z, db; int32_t beam, bin; } sonar_point;
typedef struct { float re, im; } sonar_cf32;
typedef void *sonar_stream;

/* Optional per-ray record, device arrays of [n_rays][max_bounces] with
 * n_rays = beams * rays_per_beam in (beam, ray) order: hit triangle (-1 none),
 * range bin (-1 none), connection visibility (1 visible), and contribution;
 * `stats` (optional, [n_rays][3]) receives, over all of the ray's traversals,
 * the internal nodes visited, the triangles tested and the deepest traversal
 * stack. Counting uses separate kernel instantiations: indices and bins are
 * the same as without it, values the same up to rounding. `beam` (optional,
 * [n_rays][max_bounces]) receives the beam each contribution is added to
 * (the launch beam unless SONAR_FLAG_RX_BEAMS moves it). `retro_bin` and
 * `retro_amp` (optional, [n_rays][max_bounces]) receive each vertex's
 * retro-chain return under SONAR_FLAG_RETRO_CHAIN (bin -1: none; vertex 0
 * never has one). */
typedef struct {
    int32_t *tri;
    int32_t *bin;
    int32_t *vis;
    sonar_cf32 *amp;
    uint32_t *stats;
    int32_t *beam;
    int32_t *retro_bin;
    sonar_cf32 *retro_amp;
} sonar_ray_record;

typedef struct {
    int64_t n_triangles;
    int64_t n_nodes;        /* 4-wide hierarchy nodes (128 bytes each) */
    int32_t depth;          /* levels of 4-wide nodes (a traversal stack needs at most 3 per level) */
    int32_t leaf_size;
    float lo[3], hi[3];     /* scene bounding box */
    int64_t node_bytes;     /* bytes of the node array */
    int64_t tri_bytes;      /* bytes of the triangle array */
} sonar_scene_info;

/* Builds the scene a ping traces (Sec. II-B: the simulation engine supplies
 * the geometry and per-material metadata; Sec. II-A: rays are cast in
 * parallel through it): the triangle records with their reflectivity, phase
 * and material, and the ray-traversal hierarchy (linear BVH: Morton codes of
 * triangle centroids, radix sort, binary radix tree, bottom-up bounds, then
 * 4-wide nodes collapsed greedily by surface area: a node opens its largest
 * non-leaf child until it has four).
 * Synchronous on `stream`. Returns SONAR_E_INVALID for null pointers,
 * n_triangles < 1 or >= 2^28, indices out of range or non-finite vertices
 * (checked on the device, reported after the build's synchronisation), and
 * SONAR_E_UNSUPPORTED for a hierarchy of more than 2^25 4-wide nodes. */
sonar_status sonar_build_scene(const sonar_mesh *mesh, sonar_stream stream, sonar_scene **out);

/* Frees a scene (NULL is ignored). The caller guarantees no call using it is
 * still in flight. */
void sonar_free_scene(sonar_scene *scene);

sonar_status sonar_get_scene_info(const sonar_scene *scene, sonar_scene_info *info);

/* One ping (Sec. II-A/II-B): ray generation, nearest-hit traversal, bounce
 * continuation with connection rays, scattering, spreading, absorption and
 * phase, and coherent per-beam range accumulation.
 *   volume   device complex64 [beams_v][beams_h][n_range], fully overwritten
 *   gbuffer  optional device float32 [beams_v][beams_h][8]: over the beam's
 *            first-bounce hits in range, mean range / r_max, mean cos
 *            incidence, mean rho, mean facet normal (xyz, facing the ray),
 *            hit count / rays_per_beam, and the vertical (world z)
 *            component of the beam axis (cell centre; the grid node in
 *            grid_mode 1)
 *   incoh    optional device float32 [2][beams_v][beams_h][n_range]:
 *            sum |A|^2 of first-bounce (0) and later-bounce (1) returns
 *   record   optional per-ray record (testing)
 *   ray_mask optional device bit mask over rays (bit r of word r / 32): set
 *            rays are traced and recorded but add nothing to the outputs
 * Asynchronous on `stream`. No workspace: SONAR_FLAG_RX_BEAMS with
 * max_bounces > 1 is rejected (SONAR_E_INVALID; use sonar_ping_rx). */
sonar_status sonar_ping(const sonar_scene *scene, const sonar_params *params, const sonar_pose *pose,
                        sonar_cf32 *volume, float *gbuffer, float *incoh, const sonar_ray_record *record,
                        const uint32_t *ray_mask, sonar_stream stream);

/* A general depth-dependent sound speed (Sec. II-A: rays bend by Snell's
 * law in a spatially varying sound-speed field): c(z) piecewise linear
 * through n_knots knots (z[k], c[k]), z strictly increasing, c > 0; the
 * first and last layers extend below z[0] and above z[n-1]. Inside a layer
 * a ray is that layer's circle; at a knot it continues with the same
 * direction (c is continuous) and the next curvature. */
#define SONAR_MAX_SSP_KNOTS 8
typedef struct {
    int32_t n_knots, pad;
    double z[SONAR_MAX_SSP_KNOTS];
    double c[SONAR_MAX_SSP_KNOTS];
} sonar_ssp;

/* sonar_ping through a piecewise-linear sound-speed profile (params->c0 and
 * c_grad are replaced by it; times convert to range with c at the sensor).
 * With several bounces each later vertex returns to the sensor along its
 * first-arriving eigenray among those with at most one turning point (the
 * direct ray, or one turning above or below both ends at a depth where c
 * exceeds every speed on the way there, the turning depth searched within
 * 2 r_max); a vertex no such ray reaches (a shadow zone) returns nothing
 * (record vis 0). SONAR_E_INVALID for 2 > n_knots > SONAR_MAX_SSP_KNOTS,
 * knots not strictly increasing, c <= 0 at a knot or over the scene, and
 * for SONAR_FLAG_RX_BEAMS with max_bounces > 1 (that needs the workspace of
 * sonar_ping_ssp_rx); SONAR_E_UNSUPPORTED for layers bending more than
 * |g| 2 r_max / c = 1e-2. Asynchronous on `stream`; no workspace. */
sonar_status sonar_ping_ssp(const sonar_scene *scene, const sonar_params *params, const sonar_pose *pose,
                            const sonar_ssp *ssp, sonar_cf32 *volume, float *gbuffer, float *incoh,
                            const sonar_ray_record *record, const uint32_t *ray_mask, sonar_stream stream);

/* sonar_ping_ssp with a workspace (as sonar_ping_rx: device memory of at
 * least sonar_rx_workspace_size(params) bytes, 256-byte aligned, owned by the
 * caller, one ping at a time), for SONAR_FLAG_RX_BEAMS with several bounces
 * through the layered profile. */
sonar_status sonar_ping_ssp_rx(const sonar_scene *scene, const sonar_params *params, const sonar_pose *pose,
                               const sonar_ssp *ssp, sonar_cf32 *volume, float *gbuffer, float *incoh,
                               const sonar_ray_record *record, const uint32_t *ray_mask, void *workspace,
                               size_t ws_bytes, sonar_stream stream);

/* Bytes of device workspace sonar_ping_rx needs: a list of up to
 * n_rays * (max_bounces - 1) returns that receive binning moves to another
 * beam (16 bytes each) and its counter; 0 when the parameters are invalid. */
size_t sonar_rx_workspace_size(const sonar_params *params);

/* sonar_ping with a workspace, for SONAR_FLAG_RX_BEAMS with several
 * bounces: returns binned to another beam are listed during the ping and
 * added into that beam's column (and the bounce >= 2 incoherent channel)
 * after it, with floating-point atomics, so the order of those additions
 * and the last bits of the affected cells may vary between runs. Any other
 * parameters behave as in sonar_ping. Asynchronous on `stream`; no
 * allocation. */
sonar_status sonar_ping_rx(const sonar_scene *scene, const sonar_params *params, const sonar_pose *pose,
                           sonar_cf32 *volume, float *gbuffer, float *incoh, const sonar_ray_record *record,
                           const uint32_t *ray_mask, void *workspace, size_t workspace_bytes, sonar_stream stream);

/* Bytes of device workspace a ping with a workspace (sonar_ping_ws) needs
 * for these parameters, times n_pings (one area per ping in flight at once):
 * with several bounces, the per-ray state of the staged kernels (80 bytes
 * per ray), the winner of each traversal (8 bytes per ray), the pending
 * connection queries (64 bytes per ray) and the
 * contribution slots (20 bytes per ray and contribution: K, or 2K - 1 with
 * retro-chain returns; plus 4 bytes per ray and bounce for receive beams),
 * and the receive-binning list when SONAR_FLAG_RX_BEAMS needs it. 0 for a
 * single bounce without receive binning (no workspace needed), for a null
 * scene, n_pings < 1 or invalid parameters. */
size_t sonar_workspace_size(const sonar_scene *scene, const sonar_params *params, int32_t n_pings);

/* sonar_ping with a workspace (device memory of at least
 * sonar_workspace_size(scene, params, 1) bytes, 256-byte aligned, owned by
 * the caller, one ping at a time per area). With several bounces the ping
 * runs in stages (Sec. II-B: a bounded number of secondary reflections):
 * each bounce's nearest-hit traversal and each return path's visibility
 * traversal is a kernel over all rays, the FP64 ray state passing between
 * them through the workspace, and a last kernel reduces the contributions
 * into the columns in the fixed order of sonar_ping: records are identical
 * and volumes equal up to FP32 rounding. A request for traversal counters
 * (record->stats) runs the fused kernel. Otherwise as sonar_ping (and
 * sonar_ping_rx for receive binning). Asynchronous on `stream`; no
 * allocation. */
sonar_status sonar_ping_ws(const sonar_scene *scene, const sonar_params *params, const sonar_pose *pose,
                           sonar_cf32 *volume, float *gbuffer, float *incoh, const sonar_ray_record *record,
                           const uint32_t *ray_mask, void *workspace, size_t workspace_bytes, sonar_stream stream);

/* Bytes of device workspace sonar_detect needs for these parameters; with
 * several bounces it also holds the receive-binning list (with
 * SONAR_FLAG_RX_BEAMS) and the staged kernels' buffers, so that
 * sonar_ping_detect runs the staged ping (a smaller workspace that still
 * holds the detection and list areas runs the fused kernel). */
size_t sonar_detect_workspace_size(const sonar_params *params);

/* Per-beam CA-CFAR detection of a volume into a point cloud (Sec. II-A: an
 * azimuth-elevation-range point cloud). Power P = |E|^2 + noise_floor;
 * a cell is detected when P exceeds alpha(N) times the mean of its N training
 * cells (alpha(N) = N (pfa^(-1/N) - 1)), exceeds its lower neighbour and is
 * not below its upper one. The `max_per_beam` strongest per beam (ties: lower
 * range) are emitted in (beam, range) order at the beam centre along a
 * straight line at the bin-centre range, with 10 log10 P in dB.
 *   points     device sonar_point [capacity]
 *   dev_count  device int32[1]: total number of detections (may exceed
 *              capacity; only `capacity` are written)
 *   workspace  device buffer of sonar_detect_workspace_size() bytes
 * Asynchronous on `stream`. */
sonar_status sonar_detect(const sonar_cf32 *volume, const sonar_params *params, const sonar_pose *pose,
                          const sonar_cfar *cfar, sonar_point *points, int32_t capacity, int32_t *dev_count,
                          void *workspace, size_t workspace_bytes, sonar_stream stream);

/* One ping followed by detection, as sonar_ping then sonar_detect, with the
 * CFAR test evaluated inside the ping kernel while each beam's column is
 * still indexed on chip, so the volume is written once and never re-read.
 * Outputs and workspace as for sonar_ping (volume) and sonar_detect (points,
 * dev_count, workspace). Points are identical to sonar_detect's on the same
 * volume up to FP64 rounding of the training sums. When some alpha(N) <= 1
 * (pfa above about 0.37) a bin without a return could be detected; the call
 * then runs the two stages separately. Asynchronous on `stream`. */
sonar_status sonar_ping_detect(const sonar_scene *scene, const sonar_params *params, const sonar_pose *pose,
                               const sonar_cfar *cfar, sonar_cf32 *volume, sonar_point *points, int32_t capacity,
                               int32_t *dev_count, void *workspace, size_t workspace_bytes, sonar_stream stream);

/* sonar_ping_detect without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation). The detection workspace (and, for receive
 * binning with several bounces, the list of moved returns) lives in a
 * static device array of SONAR_NOALLOC_SCRATCH_BYTES that the library holds
 * on every GPU it runs on until the process ends; the call itself allocates
 * nothing. Outputs, results and asynchrony as sonar_ping_detect (identical
 * volume bits and points). Every call on one GPU shares that GPU's array
 * and leaves its contents behind (nothing in it needs clearing: each call
 * writes what it reads), so calls that overlap in time on one GPU (on
 * several streams, or from several threads without ordering) race and must
 * be serialised by the caller. The scene's device must be current.
 * SONAR_E_INVALID when the parameters need more scratch than the array holds
 * (about 63,000 beams without receive binning) or for any argument
 * sonar_ping_detect rejects; SONAR_E_DEVICE if the array's address cannot
 * be resolved. */
#define SONAR_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
sonar_status sonar_ping_detect_noalloc(const sonar_scene *scene, const sonar_params *params, const sonar_pose *pose,
                                       const sonar_cfar *cfar, sonar_cf32 *volume, sonar_point *points,
                                       int32_t capacity, int32_t *dev_count, sonar_stream stream);

/* ---------------------------------------------------------------------- */
/* Water-column volume reverberation and receiver noise (Sec. II-B names
 * scattering within the water volume and speckle as extensions). Every range
 * cell (beam b = v * n_h + h, bin n) of cell-centred beams holds unresolved
 * scatterers: its echo is a circular complex Gaussian of mean power
 *   P = s_v V / r^4 10^(-abs_db_per_m 2 r / 10) + noise_power,
 * r = r_min + (n + 1/2) dr, V = r^2 cos(el_v) dth_h dth_v dr the cell volume
 * (el_v the row's centre elevation), s_v = 10^(sv_db / 10) in 1/m. The
 * sample sqrt(P / 2) sqrt(-2 ln u1) exp(2 pi i u2) is added to the cell, with
 * u1 = ((z >> 40) + 1) / 2^24, u2 = ((z >> 16) mod 2^24) / 2^24 and
 * z = SplitMix64 output number c + 1 of `seed`, c = (pose->ping << 43) xor
 * (b << 12) xor n: fixed by the indices, reproducible in any order. The water
 * behind the first surface is not shadowed. */
typedef struct {
    double sv_db;            /* volume scattering strength S_v (dB re 1/m) */
    double noise_power;      /* receiver noise power per cell, >= 0 */
    uint64_t seed;
} sonar_reverb;

/* Adds reverberation and noise to a ping's volume in place.
 *   volume  device complex64 [beams_v][beams_h][n_range] of these params
 * SONAR_E_INVALID for bad params, pose or settings (non-finite sv_db,
 * negative noise); SONAR_E_UNSUPPORTED for grid_mode 1. Asynchronous on
 * `stream`; no allocation. */
sonar_status sonar_add_reverb(sonar_cf32 *volume, const sonar_params *params, const sonar_pose *pose,
                              const sonar_reverb *reverb, sonar_stream stream);

/* ---------------------------------------------------------------------- */
/* Time series and matched filtering (Sec. II-B: time-series data next to the
 * intensity volumes, so that matched filtering can be applied). A beam's
 * complex range column x[n] is read as the scene's impulse response sampled
 * at the bins' two-way delay spacing dt = 2 dr / c_ref (dr the bin width,
 * c_ref the sound speed at the sensor); p[0..L-1] is the transmitted baseband
 * pulse at that spacing. */

#define SONAR_MAX_PULSE_TAPS 64
#define SONAR_MAX_PULSE_BINS 2048

/* Two-way delay spacing of a ping's range bins (the time axis its volume
 * columns sample): dt = 2 dr / c_ref, dr = (r_max - r_min) / n_range, with
 * c_ref the sound speed at the sensor depth that converts travel time to
 * range in the ping (c0 + c_grad z_sensor, or the layered profile `ssp` at
 * z_sensor when it is not NULL).
 *   dt  host double, receives the spacing (s)
 * SONAR_E_INVALID for invalid parameters, pose or profile, a non-positive
 * speed at the sensor, or dt NULL. Host only. */
sonar_status sonar_pulse_dt(const sonar_params *params, const sonar_pose *pose, const sonar_ssp *ssp, double *dt);

/* Baseband linear-FM pulse of bandwidth B over `duration`:
 * L = max(1, round(duration / dt)) samples at t_k = (k + 1/2) dt - L dt / 2,
 * p[k] = w[k] exp(i pi (B / duration) t_k^2), with w = 1 (window 0) or
 * w[k] = sin^2(pi (k + 1/2) / L) (window 1, Hann).
 *   taps  host sonar_cf32 [max_len]; *len receives L
 * SONAR_E_INVALID for bandwidth < 0, duration <= 0, dt <= 0, another window,
 * null pointers, or L above max_len or SONAR_MAX_PULSE_TAPS. Host only. */
sonar_status sonar_lfm_pulse(double bandwidth_hz, double duration_s, double dt_s, int32_t window, sonar_cf32 *taps,
                             int32_t max_len, int32_t *len);

/* Pulse compression of n_beams complex columns of n_bins samples each:
 *   series[b][n]  = sum_{k<L} p[k] x[b][n-k]
 *   matched[b][n] = sum_{k<L} conj(p[k]) series[b][n+k]
 * with x and series zero outside [0, n_bins) (records of n_bins samples).
 *   volume   device complex64 [n_beams][n_bins], e.g. a ping's volume
 *   pulse    host complex64 [pulse_len], 1 <= pulse_len <= SONAR_MAX_PULSE_TAPS;
 *            copied into the launch, so the call allocates nothing and can be
 *            captured in a graph
 *   series   optional device complex64 [n_beams][n_bins]
 *   matched  optional device complex64 [n_beams][n_bins]
 * At least one output; the outputs must not overlap the input or each other.
 * 1 <= n_bins <= SONAR_MAX_PULSE_BINS, 0 <= n_beams < 2^31 (0: nothing).
 * Asynchronous on `stream`. */
sonar_status sonar_pulse_compress(const sonar_cf32 *volume, int64_t n_beams, int32_t n_bins, const sonar_cf32 *pulse,
                                  int32_t pulse_len, sonar_cf32 *series, sonar_cf32 *matched, sonar_stream stream);

/* ---------------------------------------------------------------------- */
/* Batches: hundreds of pings with their own poses, beam layouts and rays per
 * beam in one persistent launch. Work items are (ping, tile of 256 rays);
 * persistent workgroups pop them from one device counter. All pings of a
 * batch share the scene, max_bounces and the medium type (c_grad zero or
 * not, or one layered profile). */

/* Host summary of a prepared batch (filled by sonar_batch_prepare): `arc`
 * is the medium type, 0 straight rays, 1 one gradient, 2 a layered profile;
 * `retro` is 1 when the pings take retro-chain returns, `rx` the number of
 * pings with receive-binning lists. */
typedef struct {
    int32_t n_pings, max_bounces, arc, max_bins, max_beams, retro, rx;
    int64_t total_tiles, total_rays;
} sonar_batch_plan;

/* Launch knobs: persistent workgroups per compute unit (0: the occupancy
 * limit), work units taken per queue pop (0: 1), and the workgroup size in
 * 64-lane waves, 1, 2 or 4 (0: 4), which is also the unit of work: a unit is
 * that many waves of consecutive rays of one ping (batches through a
 * layered profile or with retro-chain returns always run 4). `emit_desc`:
 * device copy of the emission descriptors of sonar_batch_prepare_detect, or
 * NULL for a batch without detection. */
typedef struct {
    int32_t blocks_per_cu, tiles_per_item;
    const void *emit_desc;
    int32_t waves_per_block, pad;
} sonar_batch_options;

typedef struct sonar_graph sonar_graph;   /* an instantiated HIP graph of one batch */

/* Bytes of one ping descriptor (device-side argument block). */
size_t sonar_batch_desc_bytes(void);

/* Bytes of batch workspace for n_pings (queue counter and per-ping device
 * clock stamps). */
size_t sonar_batch_workspace_size(int32_t n_pings);

/* Fills n_pings descriptors into the host buffer `host_desc`
 * (n_pings * sonar_batch_desc_bytes() bytes) from per-ping parameters, poses
 * and device output volumes (volumes[i]: complex64 of ping i's layout), and
 * the plan. The caller copies host_desc to device memory; the descriptors may
 * be rewritten there between launches (new poses) as long as each ping keeps
 * its layout. SONAR_E_INVALID if pings disagree on max_bounces or medium
 * type, or any parameter fails sonar_ping's validation. */
sonar_status sonar_batch_prepare(const sonar_scene *scene, int32_t n_pings, const sonar_params *params,
                                 const sonar_pose *poses, sonar_cf32 *const *volumes, void *host_desc,
                                 sonar_batch_plan *plan);

/* sonar_batch_prepare for pings through one layered sound-speed profile (as
 * sonar_ping_ssp; each ping's time-to-range speed is c at its own sensor
 * depth). Validation as sonar_ping_ssp per ping. */
sonar_status sonar_batch_prepare_ssp(const sonar_scene *scene, int32_t n_pings, const sonar_params *params,
                                     const sonar_pose *poses, const sonar_ssp *ssp, sonar_cf32 *const *volumes,
                                     void *host_desc, sonar_batch_plan *plan);

/* Bytes of device workspace for the receive-binning lists of a batch
 * (pings with SONAR_FLAG_RX_BEAMS and several bounces; 0 when none, or when
 * a parameter set is invalid). */
size_t sonar_batch_rx_workspace_size(int32_t n_pings, const sonar_params *params);

/* sonar_batch_prepare (ssp NULL) or sonar_batch_prepare_ssp (one layered
 * profile) for batches holding pings with receive binning of several
 * bounces: each such ping gets its list area in `rx_workspace` (device, at
 * least sonar_batch_rx_workspace_size bytes, 256-byte aligned, owned by the
 * caller, one batch run at a time). sonar_ping_batch then clears the lists
 * before the pings and adds them into the volumes after them with
 * floating-point atomics (the last bits of the affected cells may vary
 * between runs). The other prepare calls reject such pings. */
sonar_status sonar_batch_prepare_rx(const sonar_scene *scene, int32_t n_pings, const sonar_params *params,
                                    const sonar_pose *poses, const sonar_ssp *ssp, sonar_cf32 *const *volumes,
                                    void *rx_workspace, size_t rx_ws_bytes, void *host_desc,
                                    sonar_batch_plan *plan);

/* Optional outputs of one ping of a prepared batch, as sonar_ping takes them
 * (Sec. II-B: the per-beam G-buffer and incoherent channels, for training
 * data; the record and ray mask, for testing): amends descriptor `ping` of
 * the n_pings descriptors in the host buffer `host_desc` (filled by
 * sonar_batch_prepare*). gbuffer, incoh, record arrays and ray_mask are
 * device pointers laid out for that ping's layout as for sonar_ping, or NULL
 * (that output off). Copy the descriptors to the device again afterwards.
 * SONAR_E_INVALID for a null host_desc, ping outside [0, n_pings), a
 * partial record or a descriptor not filled by a prepare call;
 * SONAR_E_UNSUPPORTED for record->stats (batches keep no counters). */
sonar_status sonar_batch_set_outputs(void *host_desc, int32_t n_pings, int32_t ping, float *gbuffer, float *incoh,
                                     const sonar_ray_record *record, const uint32_t *ray_mask);

/* Detection for a prepared batch (Sec. II-A: each ping's point cloud):
 * amends the ping descriptors in `host_desc` (as filled by
 * sonar_batch_prepare) so that every ping's kernel runs the CA-CFAR test of
 * sonar_ping_detect on its beams, and fills one emission descriptor per ping
 * (`host_emit`, n_pings * sonar_batch_emit_desc_bytes() bytes) for the
 * batched point emission that sonar_ping_batch then runs after the pings.
 * Per ping i: points[i] with room for capacity[i] points, its point count at
 * dev_counts[i] (device int32, written by the emission), and a detection
 * workspace slice of `workspace` (device, sonar_batch_detect_workspace_size
 * bytes in total). Copy both descriptor arrays to the device again and pass
 * the emission copy as options->emit_desc. SONAR_E_UNSUPPORTED if some
 * training-window size has alpha(N) <= 1 (the fused test would then miss
 * detections in bins without a return). */
size_t sonar_batch_emit_desc_bytes(void);
size_t sonar_batch_detect_workspace_size(int32_t n_pings, const sonar_params *params);
sonar_status sonar_batch_prepare_detect(int32_t n_pings, const sonar_params *params, const sonar_pose *poses,
                                       const sonar_cfar *cfar, sonar_point *const *points,
                                       const int32_t *capacity, int32_t *dev_counts, void *workspace,
                                       size_t workspace_bytes, void *host_desc, void *host_emit);

/* Runs a prepared batch: a reset kernel, the persistent ping kernel, and,
 * when options->emit_desc is set, one point-emission launch for all pings.
 * `dev_desc` are the descriptors in device memory. Allocates nothing, so it
 * can be captured in a graph. Asynchronous on `stream`. */
sonar_status sonar_ping_batch(const sonar_scene *scene, const sonar_batch_plan *plan, const void *dev_desc,
                              const sonar_batch_options *options, void *workspace, size_t workspace_bytes,
                              sonar_stream stream);

/* Copies the per-ping first-start and last-finish device clock stamps
 * (100 MHz constant clock, s_memrealtime) of the last batch run on
 * `workspace` into host arrays; synchronises `stream`. */
sonar_status sonar_batch_stamps(const void *workspace, int32_t n_pings, uint64_t *start, uint64_t *finish,
                                sonar_stream stream);

/* Captures one batch launch (reset + persistent kernel) into a HIP graph and
 * instantiates it; sonar_graph_launch replays it on any stream. The graph
 * keeps the descriptor and workspace pointers: update descriptors in place. */
sonar_status sonar_batch_graph_create(const sonar_scene *scene, const sonar_batch_plan *plan, const void *dev_desc,
                                      const sonar_batch_options *options, void *workspace, size_t workspace_bytes,
                                      sonar_graph **out);
sonar_status sonar_graph_launch(sonar_graph *graph, sonar_stream stream);
void sonar_graph_free(sonar_graph *graph);

/* Measures the batch under every launch-knob candidate with device events
 * (mean of three runs after a warm-up) and returns the fastest in `best`
 * (emit_desc NULL) and its time in `best_ms`. Candidates: workgroups of 1, 2
 * or 4 waves (4 only for layered or retro-chain batches) x persistent
 * workgroups per compute unit giving 1, 2, ... up to the occupancy limit of
 * waves per SIMD x units per pop in {1, 2, 4}. When the environment variable
 * SONAR_AUTOTUNE_CACHE names a file, a result cached there for the same
 * device, scene size and plan is returned without measuring; otherwise every
 * candidate's time ("cand" lines) and the choice are appended to it.
 * Synchronous. */
sonar_status sonar_batch_autotune(const sonar_scene *scene, const sonar_batch_plan *plan, const void *dev_desc,
                                  void *workspace, size_t workspace_bytes, sonar_stream stream,
                                  sonar_batch_options *best, float *best_ms);

/* ---------------------------------------------------------------------- */
/* Learned multipath surrogate (Sec. II-B: scattering functions may be learned
 * from data). A network maps each beam's single-bounce G-buffer (a 3 x 3 beam
 * neighbourhood of its 8 features) and the beam's geometry to 64
 * standardised orthonormal DCT-II coefficients of the level profile of what
 * later bounces add:
 *   lev[r] = 10 log10(1 + Ims[r] / 1e-11),
 * where Ims is the later-bounce incoherent channel of a multi-bounce ping
 * box-averaged over `smooth` range bins ([r - smooth/2, r + smooth/2)), shifted
 * so that the beam's first-hit bin (its G-buffer mean first-bounce range) is
 * bin 0, zero past the end. The predicted profile adds that intensity back:
 *   profile[r] = 10 log10(I1s[r] + 1e-11 * 10^(lev[r] / 10)),
 * so a zero level leaves the smoothed single-bounce profile.
 * Geometry of a beam, from its image's geometry block (16 floats: sensor
 * position, the sensor-to-world rotation row-major, hfov, vfov, two zeros;
 * sonar_surrogate_geometry fills one) and its G-buffer entry: the beam axis u
 * in the world (cell-centred beams: azimuth -hfov/2 + (h + 1/2) hfov / W,
 * elevation -vfov/2 + (v + 1/2) vfov / H), the mean first hit on it P = S +
 * r_max g0 u (the origin for a beam without hits, g6 = 0), the axis mirrored
 * at the mean first-hit normal n = (g3, g4, g5), m = u - 2 (u . n) n / |n|^2
 * (zero without a hit or a normal), and 102 columns: P / 10, u, S / 10, m
 * (lengths in metres), then sin(pi/2 2^k x) for the nine values x of P / 10,
 * u and m (x-major, k = 0 .. 4), then the cosines. Later bounces go where
 * the scene sends the continuation of the first hit: for one scene the
 * network learns that from where the hit is and where it sends the
 * continuation.
 * Layers: the 72 neighbourhood columns (an im2col product) and the 102
 * geometry columns -> 64, then 64 -> 256 -> 256 -> 256 -> 64, ReLU between
 * layers; 175,872 parameters.
 * Products use BF16 operands on the matrix cores with FP32 accumulation;
 * training is a weighted MSE on the coefficients, sum_j w_j (y_j - t_j)^2 over
 * rows * 64 (weights 1 by default), with Adam (beta 0.9 / 0.999, eps 1e-8) on
 * FP32 master weights.
 *
 * Parameter vector layout (float, sonar_surrogate_param_count() entries): for
 * each layer W [fan_in][fan_out] row-major then b [fan_out], with (fan_in,
 * fan_out) = (174, 64), (64, 256), (256, 256), (256, 256), (256, 64); input
 * column order: the neighbourhood (dv, dh, feature), then the geometry.
 * G-buffer: float [n_img][H][W][8] as sonar_ping writes it (16-byte aligned); geometry: float
 * [n_img][16] on the device; rows = n_img * H * W (a multiple of 64 for the
 * network, at most max_rows everywhere).
 * Standardisation: coefficient j is (c_j - mean_j) / std_j (defaults 0, 1). */
typedef struct sonar_surrogate sonar_surrogate;

int64_t sonar_surrogate_param_count(void);

/* Allocates weights, Adam state, activations and smoothing buffers for up to
 * max_rows beams, and the DCT basis for n_bins range bins over [r_min, r_max)
 * (64 <= n_bins <= 2048); `smooth` is the range box width in bins. Weights start at
 * zero: set them. */
sonar_status sonar_surrogate_create(int64_t max_rows, int32_t n_bins, double r_min, double r_max, int32_t smooth,
                                    sonar_surrogate **out);
void sonar_surrogate_free(sonar_surrogate *s);

/* Host copies of the FP32 master weights and Adam moments (any may be NULL)
 * and the step count: a checkpoint. set_state with m = v = NULL resets Adam.
 * Both synchronise. */
sonar_status sonar_surrogate_set_state(sonar_surrogate *s, const float *params, const float *adam_m,
                                       const float *adam_v, int64_t step);
sonar_status sonar_surrogate_get_state(const sonar_surrogate *s, float *params, float *adam_m, float *adam_v,
                                       int64_t *step);

/* Coefficient standardisation (host arrays of 64). */
sonar_status sonar_surrogate_set_norm(sonar_surrogate *s, const float *mean, const float *std);

/* Loss weights w_j (host array of 64, finite and >= 0; NULL restores 1).
 * With w_j = std_j^2 / mean(std^2) the loss is, by Parseval's theorem, the
 * squared error of the truncated level profile itself. */
sonar_status sonar_surrogate_set_loss_weights(sonar_surrogate *s, const float *w);

/* Host: the geometry block of one ping (16 floats) from its sensor
 * parameters and pose. SONAR_E_UNSUPPORTED for the LiDAR grid (grid_mode 1),
 * SONAR_E_INVALID for null pointers or non-positive fields of view. */
sonar_status sonar_surrogate_geometry(const sonar_params *params, const sonar_pose *pose, float block[16]);

/* Inference: standardised coefficients [rows][64] (device) from a G-buffer
 * and the images' geometry blocks (device). */
sonar_status sonar_surrogate_forward(sonar_surrogate *s, const float *gbuffer, const float *geometry, int32_t n_img,
                                     int32_t h, int32_t w, float *coef, sonar_stream stream);

/* One training step on (G-buffer, geometry, standardised target
 * [rows][64]): forward, MSE, backward, Adam with learning rate lr. The loss
 * before the update goes to dev_loss (device float). */
sonar_status sonar_surrogate_train_step(sonar_surrogate *s, const float *gbuffer, const float *geometry, int32_t n_img,
                                        int32_t h, int32_t w, const float *target, float lr, float *dev_loss,
                                        sonar_stream stream);

/* Gradient of the MSE w.r.t. the parameter vector (device float
 * [param_count]) without updating; for checks. */
sonar_status sonar_surrogate_gradient(sonar_surrogate *s, const float *gbuffer, const float *geometry, int32_t n_img,
                                      int32_t h, int32_t w, const float *target, float *dev_grad, float *dev_loss,
                                      sonar_stream stream);

/* Level target: coefficients [rows][64] from the later-bounce incoherent
 * channel im [rows][n_bins] and the G-buffer of the same beams (device),
 * standardised when `standardize` is 1. */
sonar_status sonar_surrogate_target(const sonar_surrogate *s, const float *im, const float *gbuffer, int64_t rows,
                                    int32_t standardize, float *coef, sonar_stream stream);

/* Sums of the 64 coefficients and of their squares over rows (host double
 * arrays of 64), for the standardisation statistics. Synchronises. */
sonar_status sonar_surrogate_moments(sonar_surrogate *s, const float *coef, int64_t rows, double *sum, double *sum_sq,
                                     sonar_stream stream);

/* Predicted multi-bounce profile and its errors. For standardised
 * predictions `coef`: profile[r] = 10 log10(I1[r] + 1e-11 * 10^(lev[r] / 10))
 * at full range resolution, with I1 the single-bounce channel as given and
 * lev the inverse DCT of the de-standardised coefficients from the first-hit
 * bin on and 0 before it (written to `profile` [rows][n_bins] if not NULL).
 * If `im` is not NULL, `err` [rows][8] receives per beam mean |error| in dB
 * (NaN when no bin counts):
 *   the range-smoothed prediction 10 log10(I1s + 1e-11 * 10^(lev / 10)) over
 *   bins whose smoothed truth 10 log10(I1s + Ims + 1e-11) is more than 3 dB
 *   above the floor: [0] the prediction, [1] the smoothed single bounce,
 *   [2] the smoothed single bounce plus the mean level (inverse DCT of the
 *   mean coefficients), [3] the number of such bins;
 *   the full-resolution profile over bins whose raw truth
 *   10 log10(I1 + Im + 1e-11) is more than 3 dB above the floor: [4] the
 *   prediction, [5] the single bounce plus the mean level, [6] the single
 *   bounce 10 log10(I1 + 1e-11), [7] the number of such bins. */
sonar_status sonar_surrogate_profile(const sonar_surrogate *s, const float *coef, const float *i1, const float *im,
                                     const float *gbuffer, int64_t rows, float *profile, float *err,
                                     sonar_stream stream);

/* Synchronises `stream` and reports device-side errors recorded by calls
 * that used `scene` (SONAR_E_STACK if a traversal ran out of stack). Clears
 * the record. */
sonar_status sonar_device_status(const sonar_scene *scene, sonar_stream stream);

/* Static description of a status code. */
const char *sonar_status_string(sonar_status status);

/* Detail of the last failure on the calling thread ("" if none). */
const char *sonar_last_error(void);

/* Sec. III, Eq. (1)-(3): fills n_range, n_h, n_v (and hfov, vfov, r_min,
 * r_max) of `params` from fields of view (rad), angular resolutions (rad),
 * range limits and range resolution (m), as floor() of each quotient (with a
 * 1e-9 guard for quotients that are integers in exact arithmetic). Other
 * fields are left unchanged. */
sonar_status sonar_params_from_resolution(double hfov, double vfov, double dth_h, double dth_v, double r_min,
                                          double r_max, double dr, sonar_params *params);

#ifdef __cplusplus
}
#endif

#endif /* SONAR_H */
