// Internal types shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sonar.h"

namespace sonar {

// ---------------------------------------------------------------------------
// Scene layout in HBM.
//
// Node: 64 bytes, two child boxes and two child links:
//   float4 a = {lo0.x, lo0.y, lo0.z, hi0.x}
//   float4 b = {hi0.y, hi0.z, lo1.x, lo1.y}
//   float4 c = {lo1.z, hi1.x, hi1.y, hi1.z}
//   int4   d = {link0, link1, 0, 0}
// Link: >= 0 internal node index; LEAF_BIT | first << 3 | (count - 1) a leaf of
// `count` consecutive triangle records; EMPTY_LINK no child.
// Triangle record: 48 bytes, the FP32 input vertices (exact), the original
// triangle index with the pressure-release bit, reflectivity and phase:
//   float4 {v0.x, v0.y, v0.z, v1.x}, {v1.y, v1.z, v2.x, v2.y},
//          {v2.z, bits(id | mat << 31), rho, phi}
constexpr uint32_t LEAF_BIT = 0x80000000u;
constexpr uint32_t EMPTY_LINK = 0xFFFFFFFFu;
constexpr uint32_t MAT_BIT = 0x80000000u;
constexpr int MAX_BOUNCES = 4;
constexpr int MAX_BINS = 4096;

struct Scene {
    float4 *nodes = nullptr;      // [n_nodes * 8]: 4-wide nodes of 128 bytes
    float4 *tris = nullptr;       // [n_tri * 3]
    int *status = nullptr;        // device error word
    int64_t n_tri = 0;
    int64_t n_nodes = 0;
    int depth = 0;                // levels of 4-wide nodes
    int binary_depth = 0;         // height of the binary tree they come from
    int stack = 0;                // bound on traversal stack entries (3 per level)
    int leaf_size = 4;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    float zabs_max = 0.f;
    int device = 0;
};

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output number n of the
// generator seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix64_nth(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Device status bits.
constexpr int ST_STACK = 1;
constexpr int ST_BAD_INDEX = 2;
constexpr int ST_BAD_VERTEX = 4;
constexpr int ST_BAD_TREE = 8;
constexpr int ST_LOOP = 16;
constexpr int ST_RX_FULL = 32;

// Everything a ping kernel needs, by value.
constexpr uint32_t FLAG_BEAM_PATTERN = 1u;
constexpr int MAX_SSP_KNOTS = 8;
constexpr uint32_t FLAG_RX_BEAMS = 2u;
constexpr uint32_t FLAG_DIFFUSE_BOUNCE = 4u;
constexpr uint32_t FLAG_RETRO_CHAIN = 8u;

// Staged multi-bounce ping: what one bounce hands to the next (FP64 origin
// and direction of the continuation, out-path length and time, path
// weight; L_out < 0 marks a ray that has stopped).
struct alignas(16) RayState {
    double o[3];
    double d[3];
    double L_out, T_out, Wt;
    uint32_t prev;       // the facet the continuation leaves from
    float w_tx;          // transmit pattern at the launch direction
};
// One traversal query in FP32 (a straight ray, or the chord of an arc with
// its tangent, centre normal, curvature and box inflation), ready for a
// traversal kernel: the continuation of a bounce or the return path of a
// vertex (visibility).
struct alignas(16) SegRec {
    float o[3], sigma;
    float d[3], tmin;
    float ad[3], tmax;
    float anc[3], kappa;
    float smin, smax;
    uint32_t skip;       // the facet the query leaves from (never reported)
    int32_t live;        // 0: nothing to trace
};

struct PingArgs {
    const float4 *nodes;
    const float4 *tris;
    int *status;
    // sensor
    double pos[3];
    double rot[9];
    double hfov, vfov, dth_h, dth_v;
    double r_min, r_max, dr;
    double f0, c0, g, alpha_db;
    double k_d, k_s, phong_n;
    double c_ref, c_hi;
    double tan_h, tan_v;     // tan(hfov / 2) (when hfov < pi), tan(vfov / 2)
    uint64_t seed;
    uint32_t ping;
    int beams_h, beams_v, n_beams, n_r, log2_nr, na, ne;
    int grid_mode, jitter, n_bins, K;
    int64_t n_rays;
    // outputs
    float2 *volume;
    float *gbuf;
    float *incoh;
    int32_t *rec_tri, *rec_bin, *rec_vis, *rec_beam, *rec_rbin;
    float2 *rec_amp, *rec_ramp;
    uint32_t *stats;         // optional [n_rays][3]: internal nodes visited, triangles tested, deepest stack
    const uint32_t *mask;
    uint32_t max_steps;      // node-visit bound of one traversal (2 * nodes + 64)
    // fused detection (det_count == nullptr: off)
    int32_t *det_count;      // [n_beams]
    int32_t *det_bins;       // [n_beams * det_M], strongest first
    float *det_pw;           // [n_beams * det_M]
    int det_G, det_T, det_M;
    float det_n0;
    double det_alpha[2 * 64 + 1];
    // beam forming: FLAG_BEAM_PATTERN / FLAG_RX_BEAMS; returns binned to
    // another beam go to rx_list (beam, bin, re, im) through rx_count
    // piecewise-linear sound speed (n_layers > 0): knots lay_z[0..n_layers],
    // layer i spans [lay_z[i], lay_z[i+1]] (the first and last extend to
    // -inf and +inf) with c = lay_c0[i] + lay_g[i] z
    int n_layers;
    double lay_z[MAX_SSP_KNOTS], lay_g[MAX_SSP_KNOTS], lay_c0[MAX_SSP_KNOTS];
    uint32_t flags;
    uint32_t rx_cap;
    int4 *rx_list;
    uint32_t *rx_count;
    // batch bookkeeping (descriptor of one ping in a batch)
    int tile_offset;         // first global tile of this ping
    int n_tiles;             // 256-ray tiles of this ping
    // staged multi-bounce path (stg_state == nullptr: the fused kernel):
    // per-ray state, connection queries, and contribution slots
    // [KS][n_rays] (bin, value) plus their receive beams [K][n_rays]
    RayState *stg_state;
    SegRec *stg_seg;         // [n_rays]: next nearest-hit query of every ray
    SegRec *stg_cseg;        // [n_rays]: return-path (visibility) query of the last bounce
    int2 *stg_hit;           // [n_rays]: winner of the last traversal (record index, FP32 arc length bits)
    int32_t *stg_bin;
    float4 *stg_val;
    int32_t *stg_rxb;
};

// One batch launch: descriptors in device memory, one kernel class.
struct DetectArgs;
struct BatchLaunch {
    const PingArgs *desc;
    int n_pings;
    int K;
    bool arc;
    bool layered;            // every ping through its layered profile (descriptors carry it)
    bool retro;              // every ping with retro-chain returns
    bool rx;                 // some ping lists returns for receive binning (clear before, scatter after)
    int depth;               // hierarchy depth (selects the stack size)
    int max_bins;            // largest n_range of the batch (LDS sizing)
    int64_t total_tiles;
    uint32_t *queue;
    unsigned long long *t0, *t1;
    int blocks_per_cu;       // persistent grid = CUs x this (0: occupancy limit)
    int tiles_per_item;      // units popped per queue operation
    int waves_per_block;     // workgroup size in waves (1, 2, 4; layered and retro batches: 4); a unit is that many 64-ray waves
    const DetectArgs *emit;  // batched point emission after the pings (nullptr: none)
    int max_beams;           // largest beam count of the batch (emission grid)
};
hipError_t launch_ping_batch(const BatchLaunch &b, hipStream_t s);
int batch_max_blocks_per_cu(const BatchLaunch &b);

// Host-side launchers (one per translation unit).
hipError_t launch_ping(const PingArgs &a, int stack_depth, hipStream_t s);
// Multi-bounce ping in stages (staged.hip): bytes of its per-ray buffers,
// their placement in a workspace area (256-byte aligned), and the launches.
size_t staged_workspace_bytes(int64_t n_rays, int K, bool retro, bool rx);
void set_staged_area(PingArgs &a, void *area);
hipError_t launch_ping_staged(const PingArgs &a, int stack_depth, hipStream_t s);
// Single-bounce ping through a piecewise-linear sound-speed profile.
hipError_t launch_ping_layered(const PingArgs &a, int stack_depth, hipStream_t s);
// Receive binning: clear the list's counter before a ping; add the listed
// returns into their beams' columns after it.
hipError_t launch_rx_reset(uint32_t *count, hipStream_t s);
hipError_t launch_rx_scatter(const PingArgs &a, hipStream_t s);

struct BuildBuffers;
sonar_status build_hierarchy(const sonar_mesh &m, hipStream_t s, Scene *out, char *err, size_t errlen);

struct DetectArgs {
    const float2 *volume;
    sonar_point *points;
    int32_t *count;
    int32_t *beam_count;     // workspace [n_beams]
    int32_t *beam_bins;      // workspace [n_beams * max_per_beam]
    float *beam_pw;          // workspace [n_beams * max_per_beam]
    int n_beams, n_bins, beams_h, grid_mode;
    int train, guard, max_per_beam, capacity;
    double pfa, noise_floor;
    double hfov, vfov, dth_h, dth_v, r_min, dr;
    double pos[3], rot[9];
    double alpha[2 * 64 + 1];   // CFAR factor alpha(N) for N training cells
};
hipError_t launch_detect(const DetectArgs &a, hipStream_t s);
hipError_t launch_emit(const DetectArgs &a, hipStream_t s);
// Point emission of a batch: descriptors in device memory, one grid row per ping.
hipError_t launch_emit_batch(const DetectArgs *dev_desc, int n_pings, int max_beams, hipStream_t s);
size_t detect_workspace_bytes(int n_beams, int max_per_beam);

// Pulse compression (pulse.hip): series and matched output of complex columns.
constexpr int MAX_PULSE_TAPS = 64;
constexpr int MAX_PULSE_BINS = 2048;
struct PulseArgs {
    const float2 *x;         // [n_beams][n_bins]
    float2 *s;               // series, or nullptr
    float2 *y;               // matched output, or nullptr
    int64_t n_beams;
    int n_bins, L;
    float2 p[MAX_PULSE_TAPS];
};
hipError_t launch_pulse(const PulseArgs &a, hipStream_t s);

// Volume reverberation and receiver noise (reverb.hip).
struct ReverbArgs {
    float2 *volume;          // [n_beams][n_bins], updated in place
    int64_t n_beams;
    int n_bins, beams_h;
    float r_min, dr, vfov, dth_v, cell_solid;   // cell_solid = dth_h * dth_v
    float sv, alpha_db, noise;
    uint64_t seed;
    uint32_t ping;
};
hipError_t launch_reverb(const ReverbArgs &a, hipStream_t s);

}  // namespace sonar
