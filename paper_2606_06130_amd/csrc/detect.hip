// Per-beam detection of a complex range volume into a point cloud (Sec. II-A:
// the volumetric sensor's output as an azimuth-elevation-range point cloud).
// Cell-averaging CFAR (Finn and Johnson, 1968): alpha(N) = N (pfa^(-1/N) - 1)
// times the mean of the N training cells, a local-peak test, the strongest
// `max_per_beam` cells per beam, then a deterministic (beam, range) ordering
// through an exclusive scan of the per-beam counts.
//
// k_cfar: one 256-thread block per beam. The column is read once with
// coalesced 16-byte loads, powers go to LDS, an FP64 block prefix sum gives
// every training window in four LDS reads, and alpha(N) comes from a table
// built on the host. HBM traffic: the volume, once.
// k_emit: one thread per beam, 256 beams per block; the block's offset is the
// sum of all earlier counts (read from L2), then a block scan places its
// points in (beam, range) order.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.hpp"

namespace sonar {

namespace {

constexpr int CT = 256;                 // k_cfar threads
constexpr int CW = CT / 64;             // k_cfar waves
constexpr int ET = 256;                 // k_emit threads = beams per k_emit block

__device__ __forceinline__ uint64_t pack_key(float p, int r)
{
    // larger power first, then lower range: compare (power bits, ~range)
    return ((uint64_t)__float_as_uint(p) << 32) | (uint32_t)(~r);
}

// Inclusive block scan (FP64) of one value per thread.
__device__ __forceinline__ double block_scan_incl(double v, double *wsum)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        double o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    double add = 0.0;
    for (int q = 0; q < w; ++q) add += wsum[q];
    return v + add;
}

__device__ __forceinline__ int block_scan_excl_int(int v, int *wsum, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        int o = __shfl_up(x, off);
        if (lane >= off) x += o;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int add = 0, tot = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
        if (q < w) add += wsum[q];
        tot += wsum[q];
    }
    *total = tot;
    return x - v + add;
}

}  // namespace

__global__ __launch_bounds__(CT) void k_cfar(DetectArgs a)
{
    extern __shared__ double sh[];
    __shared__ double wsum[CW];
    __shared__ uint64_t wtop[CW][16];
    const int nb = a.n_bins;
    double *pre = sh;                                    // [nb + 1]
    float *pw = reinterpret_cast<float *>(sh + nb + 1);   // [nb]
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int beam = blockIdx.x;
    const float2 *col = a.volume + (size_t)beam * nb;
    const float n0 = (float)a.noise_floor;

    // coalesced load: 2 bins per 16-byte load when the column is 16-byte aligned
    if ((nb & 1) == 0) {
        const float4 *c4 = reinterpret_cast<const float4 *>(col);
        for (int i = t; i < nb / 2; i += CT) {
            float4 e = c4[i];
            pw[2 * i] = e.x * e.x + e.y * e.y + n0;
            pw[2 * i + 1] = e.z * e.z + e.w * e.w + n0;
        }
    } else {
        for (int r = t; r < nb; r += CT) {
            float2 e = col[r];
            pw[r] = e.x * e.x + e.y * e.y + n0;
        }
    }
    __syncthreads();
    // FP64 prefix sum: thread t owns a contiguous chunk
    const int chunk = (nb + CT - 1) / CT;
    const int c0 = min(t * chunk, nb), c1 = min(c0 + chunk, nb);
    double run = 0.0;
    for (int r = c0; r < c1; ++r) run += (double)pw[r];
    double incl = block_scan_incl(run, wsum);
    double acc = incl - run;
    for (int r = c0; r < c1; ++r) {
        pre[r] = acc;
        acc += (double)pw[r];
    }
    if (t == CT - 1) pre[nb] = incl;
    __syncthreads();

    // detections of this thread's bins, its M largest keys kept in order
    const int G = a.guard, T = a.train, M = a.max_per_beam;
    uint64_t mine[16];
    int have = 0;
    for (int r = t; r < nb; r += CT) {
        const float p = pw[r];
        if (r > 0 && !(p > pw[r - 1])) continue;
        if (r + 1 < nb && !(p >= pw[r + 1])) continue;
        int l0 = max(r - G - T, 0), l1 = max(r - G, 0);            // [l0, l1)
        int h0 = min(r + G + 1, nb), h1 = min(r + G + T + 1, nb);  // [h0, h1)
        int N = (l1 - l0) + (h1 - h0);
        if (N <= 0) continue;
        double sum = (pre[l1] - pre[l0]) + (pre[h1] - pre[h0]);
        double thr = a.alpha[N] * sum / N;
        if (!((double)p > thr)) continue;
        uint64_t key = pack_key(p, r);
        if (have < M) {
            int q = have++;
            while (q > 0 && mine[q - 1] < key) { mine[q] = mine[q - 1]; --q; }
            mine[q] = key;
        } else if (key > mine[M - 1]) {
            int q = M - 1;
            while (q > 0 && mine[q - 1] < key) { mine[q] = mine[q - 1]; --q; }
            mine[q] = key;
        }
    }
    // per wave: the M largest keys of its lanes (0 = none)
    int head = 0;
    for (int m = 0; m < M; ++m) {
        uint64_t my = head < have ? mine[head] : 0ull;
        uint64_t best = my;
        for (int off = 32; off > 0; off >>= 1) {
            uint64_t o = __shfl_xor(best, off);
            best = o > best ? o : best;
        }
        if (best != 0ull && my == best) ++head;
        if (lane == 0) wtop[w][m] = best;
    }
    __syncthreads();
    // wave 0 merges the per-wave lists
    if (w == 0) {
        uint64_t my = lane < CW * M ? wtop[lane / M][lane % M] : 0ull;
        int kept = 0;
        int sel = -1;
        for (int m = 0; m < M; ++m) {
            uint64_t best = my;
            for (int off = 32; off > 0; off >>= 1) {
                uint64_t o = __shfl_xor(best, off);
                best = o > best ? o : best;
            }
            if (best == 0ull) break;
            if (lane == m) sel = (int)(~(uint32_t)(best & 0xFFFFFFFFu));
            if (my == best) my = 0ull;
            ++kept;
        }
        // range order: rank of each selected bin among the kept ones
        int rank = 0;
        for (int x = 0; x < kept; ++x) {
            int other = __shfl(sel, x);
            if (lane < kept && other < sel) ++rank;
        }
        if (lane < kept) {
            a.beam_bins[(size_t)beam * M + rank] = sel;
            a.beam_pw[(size_t)beam * M + rank] = pw[sel];
        }
        if (lane == 0) a.beam_count[beam] = kept;
    }
}

__global__ __launch_bounds__(ET) void k_emit(DetectArgs a)
{
    __shared__ int wsum[ET / 64];
    __shared__ int wred[ET / 64];
    const int t = threadIdx.x;
    const int g = blockIdx.x;
    // offset of this group: all counts of earlier beams (L2-resident, int4 loads)
    const int64_t before = (int64_t)g * ET;
    int part = 0;
    const int4 *c4 = reinterpret_cast<const int4 *>(a.beam_count);
    for (int64_t i = t; i < before / 4; i += ET) {
        int4 v = c4[i];
        part += v.x + v.y + v.z + v.w;
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if ((t & 63) == 0) wred[t >> 6] = part;
    const int beam = (int)before + t;
    const int c = beam < a.n_beams ? a.beam_count[beam] : 0;
    int total;
    const int excl = block_scan_excl_int(c, wsum, &total);
    int base = 0;
    for (int q = 0; q < ET / 64; ++q) base += wred[q];
    if (g == (int)gridDim.x - 1 && t == 0) *a.count = base + total;
    if (c == 0) return;
    const int M = a.max_per_beam;
    // this beam's detections in range order
    int bins[16];
    float pws[16];
    for (int x = 0; x < c; ++x) {
        int b = a.beam_bins[(size_t)beam * M + x];
        float p = a.beam_pw[(size_t)beam * M + x];
        int q = x - 1;
        while (q >= 0 && bins[q] > b) { bins[q + 1] = bins[q]; pws[q + 1] = pws[q]; --q; }
        bins[q + 1] = b;
        pws[q + 1] = p;
    }
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
    const int off = base + excl;
    for (int x = 0; x < c; ++x) {
        int dst = off + x;
        if (dst >= a.capacity) break;
        double rr = a.r_min + (bins[x] + 0.5) * a.dr;
        sonar_point p;
        p.x = (float)(a.pos[0] + wx * rr);
        p.y = (float)(a.pos[1] + wy * rr);
        p.z = (float)(a.pos[2] + wz * rr);
        p.db = (float)(10.0 * log10((double)pws[x]));
        p.beam = beam;
        p.bin = bins[x];
        a.points[dst] = p;
    }
}

size_t detect_workspace_bytes(int n_beams, int max_per_beam)
{
    size_t nb4 = ((size_t)n_beams + 3) & ~(size_t)3;            // int4-readable counts
    size_t b = 0;
    b += sizeof(int32_t) * nb4;                                   // beam_count
    b += sizeof(int32_t) * (size_t)n_beams * max_per_beam;        // bins
    b += sizeof(float) * (size_t)n_beams * max_per_beam;          // powers
    return (b + 255) & ~(size_t)255;
}

hipError_t launch_detect(const DetectArgs &a, hipStream_t s)
{
    if (a.n_beams == 0) return hipSuccess;
    size_t shmem = sizeof(double) * (a.n_bins + 1) + sizeof(float) * a.n_bins;
    hipLaunchKernelGGL(k_cfar, dim3(a.n_beams), dim3(CT), shmem, s, a);
    return launch_emit(a, s);
}

hipError_t launch_emit(const DetectArgs &a, hipStream_t s)
{
    if (a.n_beams == 0) return hipSuccess;
    int groups = (a.n_beams + ET - 1) / ET;
    hipLaunchKernelGGL(k_emit, dim3(groups), dim3(ET), 0, s, a);
    return hipGetLastError();
}

}  // namespace sonar
