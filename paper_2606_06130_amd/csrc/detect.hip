// Per-beam detection of a complex range volume into a point cloud (Sec. II-A:
// the volumetric sensor's output as an azimuth-elevation-range point cloud).
// Cell-averaging CFAR (Finn and Johnson, 1968): alpha(N) = N (pfa^(-1/N) - 1)
// times the mean of the N training cells, a local-peak test, the strongest
// `max_per_beam` cells per beam, then a deterministic (beam, range) ordering
// through an exclusive scan of the per-beam counts.
//
// One wavefront per beam: the column is read once with coalesced loads, the
// powers live in LDS and the training sums come from an FP64 prefix sum, so
// no window is re-read from HBM.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.hpp"

namespace sonar {

namespace {

constexpr int WAVE = 64;
constexpr int SCAN_THREADS = 1024;

__device__ __forceinline__ uint64_t pack_key(float p, int r)
{
    // larger power first, then lower range: compare (power bits, ~range)
    return ((uint64_t)__float_as_uint(p) << 32) | (uint32_t)(~r);
}

}  // namespace

__global__ __launch_bounds__(WAVE) void k_cfar(DetectArgs a)
{
    extern __shared__ double sh[];
    const int nb = a.n_bins;
    double *pre = sh;                                   // [nb + 1] prefix sums
    float *pw = reinterpret_cast<float *>(sh + nb + 1); // [nb] powers
    const int lane = threadIdx.x;
    const int beam = blockIdx.x;
    const float2 *col = a.volume + (size_t)beam * nb;
    const float n0 = (float)a.noise_floor;

    // chunk of contiguous bins per lane for the prefix sum
    const int chunk = (nb + WAVE - 1) / WAVE;
    for (int r = lane; r < nb; r += WAVE) {
        float2 e = col[r];
        pw[r] = e.x * e.x + e.y * e.y + n0;
    }
    __syncthreads();
    int c0 = lane * chunk, c1 = min(c0 + chunk, nb);
    double run = 0.0;
    for (int r = c0; r < c1; ++r) run += (double)pw[r];
    // inclusive scan of chunk totals across the wave
    double incl = run;
    for (int off = 1; off < WAVE; off <<= 1) {
        double v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    double acc = incl - run;
    for (int r = c0; r < c1; ++r) {
        pre[r] = acc;
        acc += (double)pw[r];
    }
    if (lane == WAVE - 1) pre[nb] = incl;
    __syncthreads();

    // detections of this lane's bins (r = lane + 64 i), best key per lane kept in order
    const int G = a.guard, T = a.train, M = a.max_per_beam;
    uint64_t cand[16];
    int ncand = 0;
    for (int r = lane; r < nb; r += WAVE) {
        int l0 = max(r - G - T, 0), l1 = max(r - G, 0);        // [l0, l1)
        int h0 = min(r + G + 1, nb), h1 = min(r + G + T + 1, nb);  // [h0, h1)
        int N = (l1 - l0) + (h1 - h0);
        if (N <= 0) continue;
        double sum = (pre[l1] - pre[l0]) + (pre[h1] - pre[h0]);
        double alpha = N * (pow(a.pfa, -1.0 / N) - 1.0);
        double thr = alpha * sum / N;
        float p = pw[r];
        bool det = (double)p > thr;
        if (r > 0 && !(p > pw[r - 1])) det = false;
        if (r + 1 < nb && !(p >= pw[r + 1])) det = false;
        if (!det) continue;
        uint64_t key = pack_key(p, r);
        // keep this lane's M best in descending order
        if (ncand < M) {
            int t = ncand++;
            while (t > 0 && cand[t - 1] < key) { cand[t] = cand[t - 1]; --t; }
            cand[t] = key;
        } else if (key > cand[M - 1]) {
            int t = M - 1;
            while (t > 0 && cand[t - 1] < key) { cand[t] = cand[t - 1]; --t; }
            cand[t] = key;
        }
    }
    // wave-wide selection of the M best keys
    int head = 0;
    int kept = 0;
    int32_t *obin = a.beam_bins + (size_t)beam * M;
    float *opw = a.beam_pw + (size_t)beam * M;
    int sel_bins[16];
    for (int m = 0; m < M; ++m) {
        uint64_t mine = head < ncand ? cand[head] : 0ull;
        uint64_t best = mine;
        for (int off = 32; off > 0; off >>= 1) {
            uint64_t o = __shfl_xor(best, off);
            best = o > best ? o : best;
        }
        if (best == 0ull) break;
        if (mine == best) ++head;
        sel_bins[m] = (int)(~(uint32_t)(best & 0xFFFFFFFFu));
        ++kept;
    }
    if (lane == 0) {
        // range order
        for (int x = 1; x < kept; ++x) {
            int v = sel_bins[x], t = x - 1;
            while (t >= 0 && sel_bins[t] > v) { sel_bins[t + 1] = sel_bins[t]; --t; }
            sel_bins[t + 1] = v;
        }
        for (int x = 0; x < kept; ++x) {
            obin[x] = sel_bins[x];
            opw[x] = pw[sel_bins[x]];
        }
        a.beam_count[beam] = kept;
    }
}

// Exclusive scan of per-beam counts in one block; writes the total.
__global__ __launch_bounds__(SCAN_THREADS) void k_count_scan(DetectArgs a)
{
    __shared__ int part[SCAN_THREADS];
    const int t = threadIdx.x;
    const int n = a.n_beams;
    const int per = (n + SCAN_THREADS - 1) / SCAN_THREADS;
    int b0 = t * per, b1 = min(b0 + per, n);
    int s = 0;
    for (int i = b0; i < b1; ++i) s += a.beam_count[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = t > 0 ? part[t - 1] : 0;
    for (int i = b0; i < b1; ++i) {
        int c = a.beam_count[i];
        a.block_sums[i] = run;
        run += c;
    }
    if (t == SCAN_THREADS - 1) *a.count = part[SCAN_THREADS - 1];
}

__global__ void k_emit(DetectArgs a)
{
    const int beam = blockIdx.x * blockDim.x + threadIdx.x;
    if (beam >= a.n_beams) return;
    const int cnt = a.beam_count[beam];
    if (cnt == 0) return;
    const int off = a.block_sums[beam];
    const int h = beam % a.beams_h, v = beam / a.beams_h;
    double az, el;
    if (a.grid_mode == 1) {
        az = -0.5 * a.hfov + h * a.dth_h;
        el = -0.5 * a.vfov + v * a.dth_v;
    } else {
        az = -0.5 * a.hfov + (h + 0.5) * a.dth_h;
        el = -0.5 * a.vfov + (v + 0.5) * a.dth_v;
    }
    double ce = cos(el), se = sin(el), ca = cos(az), sa = sin(az);
    double dx = ce * ca, dy = ce * sa, dz = se;
    double wx = a.rot[0] * dx + a.rot[1] * dy + a.rot[2] * dz;
    double wy = a.rot[3] * dx + a.rot[4] * dy + a.rot[5] * dz;
    double wz = a.rot[6] * dx + a.rot[7] * dy + a.rot[8] * dz;
    const int M = a.max_per_beam;
    for (int x = 0; x < cnt; ++x) {
        int dst = off + x;
        if (dst >= a.capacity) break;
        int bin = a.beam_bins[(size_t)beam * M + x];
        double rr = a.r_min + (bin + 0.5) * a.dr;
        sonar_point p;
        p.x = (float)(a.pos[0] + wx * rr);
        p.y = (float)(a.pos[1] + wy * rr);
        p.z = (float)(a.pos[2] + wz * rr);
        p.db = (float)(10.0 * log10((double)a.beam_pw[(size_t)beam * M + x]));
        p.beam = beam;
        p.bin = bin;
        a.points[dst] = p;
    }
}

size_t detect_workspace_bytes(int n_beams, int max_per_beam)
{
    size_t b = 0;
    b += sizeof(int32_t) * (size_t)n_beams;                      // beam_count
    b += sizeof(int32_t) * (size_t)n_beams;                      // offsets
    b += sizeof(int32_t) * (size_t)n_beams * max_per_beam;       // bins
    b += sizeof(float) * (size_t)n_beams * max_per_beam;         // powers
    return (b + 255) & ~(size_t)255;
}

hipError_t launch_detect(const DetectArgs &a, hipStream_t s)
{
    if (a.n_beams == 0) return hipSuccess;
    size_t shmem = sizeof(double) * (a.n_bins + 1) + sizeof(float) * a.n_bins;
    hipLaunchKernelGGL(k_cfar, dim3(a.n_beams), dim3(WAVE), shmem, s, a);
    hipLaunchKernelGGL(k_count_scan, dim3(1), dim3(SCAN_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_emit, dim3((a.n_beams + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sonar
