// Per-beam detection of a complex range volume into a point cloud (Sec. II-A:
// the volumetric sensor's output as an azimuth-elevation-range point cloud).
// Cell-averaging CFAR (Finn and Johnson, 1968): alpha(N) = N (pfa^(-1/N) - 1)
// times the mean of the N training cells, a local-peak test, the strongest
// `max_per_beam` cells per beam, then a deterministic (beam, range) ordering
// through an exclusive scan of the per-beam counts.
//
// k_cfar: one wave per beam, no block barriers. Each lane holds C consecutive
// bins of the column in registers (C = n_bins / 64 rounded up to a power of
// two), so peak tests read registers and lane-edge neighbours come by
// shuffle; an FP64 wave scan of the excess power P - N0 goes to LDS, from
// which every training window is four reads (windows over bins without a
// return are then exactly N * N0). alpha(N) comes from a table built on the
// host. HBM traffic: the volume, once.
// k_emit: 256 beams per block, one thread each; the block's offset is the sum
// of all earlier counts, read by all 1024 threads of the block with eight
// independent int4 loads each (one round trip up to 32,768 beams), then a
// block scan places its points in (beam, range) order. The point lies along
// the beam centre (FP32 direction: the point itself is FP32).
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.hpp"

namespace sonar {

namespace {

constexpr int ET = 1024;                // k_emit threads: all sum earlier counts
constexpr int EB = 256;                 // beams per k_emit block (its first EB threads emit)
constexpr int TOPM = 16;                // bound on max_per_beam

// LDS index of prefix entry r: one pad double per 16 entries keeps the
// chunked writes of a wave spread over the banks
__host__ __device__ __forceinline__ int pidx(int r) { return r + (r >> 4); }

__device__ __forceinline__ uint64_t pack_key(float p, int r)
{
    // larger power first, then lower range: compare (power bits, ~range)
    return ((uint64_t)__float_as_uint(p) << 32) | (uint32_t)(~r);
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

template <int C>
__global__ __launch_bounds__(64) void k_cfar(DetectArgs a)
{
    extern __shared__ double pre[];      // exclusive prefix of P - N0, entry r at pidx(r), r = 0 .. nb
    const int nb = a.n_bins;
    const int lane = threadIdx.x;
    const int beam = blockIdx.x;
    const float2 *col = a.volume + (size_t)beam * nb;
    const float n0 = (float)a.noise_floor;
    const int c0 = lane * C;                      // this lane's bins: [c0, c0 + C) within [0, nb)

    float P[C];
    if ((C & 1) == 0 && (nb & 1) == 0) {
        // column and chunk start are 16-byte aligned; c0 + 2i < nb implies c0 + 2i + 1 < nb
        const float4 *c4 = reinterpret_cast<const float4 *>(col + c0);
#pragma unroll
        for (int i = 0; i < C / 2; ++i) {
            const float4 e = (c0 + 2 * i < nb) ? c4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            P[2 * i] = e.x * e.x + e.y * e.y + n0;
            P[2 * i + 1] = e.z * e.z + e.w * e.w + n0;
        }
    } else {
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const float2 e = (c0 + i < nb) ? col[c0 + i] : make_float2(0.f, 0.f);
            P[i] = e.x * e.x + e.y * e.y + n0;
        }
    }

    // prefix of the excess over the wave: own sum, exclusive scan, own entries
    double run = 0.0;
#pragma unroll
    for (int i = 0; i < C; ++i)
        if (c0 + i < nb) run += (double)P[i] - (double)n0;
    double incl = run;
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    double acc = __shfl_up(incl, 1);
    if (lane == 0) acc = 0.0;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        if (c0 + i < nb) {
            pre[pidx(c0 + i)] = acc;
            acc += (double)P[i] - (double)n0;
        }
    }
    if (c0 < nb && c0 + C >= nb) pre[pidx(nb)] = acc;      // the lane holding the last bin
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // local peaks of this lane's bins (at most one in two consecutive bins)
    const int G = a.guard, T = a.train, M = a.max_per_beam;
    const float p_before = __shfl_up(P[C - 1], 1);          // last bin of the previous lane
    const float p_after = __shfl_down(P[0], 1);             // first bin of the next lane
    uint64_t peaks = 0ull;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const int r = c0 + i;
        const float p = P[i];
        const float pl = i > 0 ? P[i - 1] : p_before;
        const float pr = i + 1 < C ? P[i + 1] : p_after;
        const bool pk = r < nb && (r == 0 || p > pl) && (r + 1 >= nb || p >= pr);
        if (pk) peaks |= 1ull << i;
    }
    // threshold test of the peaks
    uint64_t accepted = 0ull;
    while (peaks) {
        const int i = __builtin_ctzll(peaks);
        peaks &= peaks - 1ull;
        float p = P[0];
#pragma unroll
        for (int q = 1; q < C; ++q) p = q == i ? P[q] : p;
        const int r = c0 + i;
        const int l0 = max(r - G - T, 0), l1 = max(r - G, 0);            // [l0, l1)
        const int h0 = min(r + G + 1, nb), h1 = min(r + G + T + 1, nb);  // [h0, h1)
        const int N = (l1 - l0) + (h1 - h0);
        if (N <= 0) continue;
        const double ex = (pre[pidx(l1)] - pre[pidx(l0)]) + (pre[pidx(h1)] - pre[pidx(h0)]);
        const double thr = a.alpha[N] * ((double)N * (double)n0 + ex) / N;
        if ((double)p > thr) accepted |= 1ull << i;
    }
    const int mine_n = __popcll(accepted);
    int before = mine_n;                                     // inclusive scan of the lanes' counts
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(before, off);
        if (lane >= off) before += o;
    }
    const int total = __shfl(before, 63);
    before -= mine_n;
    int kept;
    if (total <= M) {
        // every detection is kept; lanes hold ascending bins, so lane order is range order
        kept = total;
        int dst = before;
        while (accepted) {
            const int i = __builtin_ctzll(accepted);
            accepted &= accepted - 1ull;
            float p = P[0];
#pragma unroll
            for (int q = 1; q < C; ++q) p = q == i ? P[q] : p;
            a.beam_bins[(size_t)beam * M + dst] = c0 + i;
            a.beam_pw[(size_t)beam * M + dst] = p;
            ++dst;
        }
    } else {
        // the M strongest: a descending key list per lane, then M rounds of a wave maximum
        constexpr int L = (C + 1) / 2 < TOPM ? (C + 1) / 2 : TOPM;
        uint64_t mine[L];
#pragma unroll
        for (int q = 0; q < L; ++q) mine[q] = 0ull;
        while (accepted) {
            const int i = __builtin_ctzll(accepted);
            accepted &= accepted - 1ull;
            float p = P[0];
#pragma unroll
            for (int q = 1; q < C; ++q) p = q == i ? P[q] : p;
            uint64_t k = pack_key(p, c0 + i);
#pragma unroll
            for (int q = 0; q < L; ++q) {
                if (k > mine[q]) {
                    const uint64_t t = mine[q];
                    mine[q] = k;
                    k = t;
                }
            }
        }
        int sel = -1;
        float selp = 0.f;
        for (int m = 0; m < M; ++m) {
            const uint64_t my = mine[0];
            uint64_t best = my;
            for (int off = 32; off > 0; off >>= 1) {
                const uint64_t o = __shfl_xor(best, off);
                best = o > best ? o : best;
            }
            if (my == best) {
#pragma unroll
                for (int q = 0; q + 1 < L; ++q) mine[q] = mine[q + 1];
                mine[L - 1] = 0ull;
            }
            if (lane == m) {
                sel = (int)(~(uint32_t)(best & 0xFFFFFFFFu));
                selp = __uint_as_float((uint32_t)(best >> 32));
            }
        }
        kept = M;
        // range order: rank of each selected bin among the kept ones
        int rank = 0;
        for (int x = 0; x < M; ++x) {
            const int other = __shfl(sel, x);
            if (lane < M && other < sel) ++rank;
        }
        if (lane < M) {
            a.beam_bins[(size_t)beam * M + rank] = sel;
            a.beam_pw[(size_t)beam * M + rank] = selp;
        }
    }
    if (lane == 0) a.beam_count[beam] = kept;
}

// Point emission of beam group g (EB beams) of one detection.
__device__ __forceinline__ void emit_group(const DetectArgs &a, const int g)
{
    __shared__ int wsum[ET / 64];
    __shared__ int wred[ET / 64];
    const int t = threadIdx.x;
    // offset of this group: all counts of earlier beams (L2-resident int4
    // loads, eight independent ones in flight per thread)
    const int64_t before = (int64_t)g * EB;
    const int64_t n4 = before / 4;
    int part = 0;
    const int4 *c4 = reinterpret_cast<const int4 *>(a.beam_count);
    for (int64_t i0 = t; i0 < n4; i0 += 8 * ET) {
        int4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t i = i0 + (int64_t)u * ET;
            v[u] = i < n4 ? c4[i] : make_int4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) part += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if ((t & 63) == 0) wred[t >> 6] = part;
    const int beam = (int)before + t;
    const int c = (t < EB && beam < a.n_beams) ? a.beam_count[beam] : 0;
    int total;
    const int excl = block_scan_excl_int(c, wsum, &total);
    int base = 0;
    for (int q = 0; q < ET / 64; ++q) base += wred[q];
    if ((int64_t)(g + 1) * EB >= a.n_beams && t == 0) *a.count = base + total;     // the last group
    if (t >= EB || c == 0) return;
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
    float sef, cef, saf, caf;
    sincosf((float)el, &sef, &cef);
    sincosf((float)az, &saf, &caf);
    const double dx = (double)(cef * caf), dy = (double)(cef * saf), dz = (double)sef;
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
        p.db = 10.f * log10f(pws[x]);
        p.beam = beam;
        p.bin = bins[x];
        a.points[dst] = p;
    }
}

__global__ __launch_bounds__(ET) void k_emit(DetectArgs a) { emit_group(a, blockIdx.x); }

// A batch: grid row y is ping y; groups past a ping's beams have nothing to do.
__global__ __launch_bounds__(ET) void k_emit_batch(const DetectArgs *__restrict__ desc)
{
    const DetectArgs &a = desc[blockIdx.y];
    if ((int64_t)blockIdx.x * EB >= a.n_beams) return;
    emit_group(a, blockIdx.x);
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
    const size_t shmem = sizeof(double) * (size_t)(pidx(a.n_bins) + 1);
    const int per_lane = (a.n_bins + 63) / 64;
#define SONAR_CFAR(CC) hipLaunchKernelGGL(k_cfar<CC>, dim3(a.n_beams), dim3(64), shmem, s, a)
    if (per_lane <= 1) SONAR_CFAR(1);
    else if (per_lane <= 2) SONAR_CFAR(2);
    else if (per_lane <= 4) SONAR_CFAR(4);
    else if (per_lane <= 8) SONAR_CFAR(8);
    else if (per_lane <= 16) SONAR_CFAR(16);
    else if (per_lane <= 32) SONAR_CFAR(32);
    else SONAR_CFAR(64);
#undef SONAR_CFAR
    return launch_emit(a, s);
}

hipError_t launch_emit_batch(const DetectArgs *dev_desc, int n_pings, int max_beams, hipStream_t s)
{
    if (n_pings <= 0 || max_beams <= 0) return hipSuccess;
    if (n_pings > 65535) return hipErrorInvalidValue;      // grid rows
    hipLaunchKernelGGL(k_emit_batch, dim3((unsigned)((max_beams + EB - 1) / EB), (unsigned)n_pings), dim3(ET), 0, s,
                       dev_desc);
    return hipGetLastError();
}

hipError_t launch_emit(const DetectArgs &a, hipStream_t s)
{
    if (a.n_beams == 0) return hipSuccess;
    int groups = (a.n_beams + EB - 1) / EB;
    hipLaunchKernelGGL(k_emit, dim3(groups), dim3(ET), 0, s, a);
    return hipGetLastError();
}

}  // namespace sonar
