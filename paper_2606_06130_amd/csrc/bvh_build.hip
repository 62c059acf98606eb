// Linear BVH construction on the GPU: triangle bounds -> 63-bit Morton codes
// of the centroids -> stable key/value radix sort -> binary radix tree
// (Karras, "Maximizing parallelism in the construction of BVHs, octrees and
// k-d trees", HPG 2012) -> bottom-up bounds one tree level per launch ->
// 4-wide nodes (128 bytes: the four children's box planes and links) taken
// from every second level of the binary tree, with leaf collapse.
//
// The hierarchy is only an accelerator for the nearest-hit and any-hit
// queries of Sec. II-A (rays cast in parallel through a triangle scene): any
// valid hierarchy gives the same hits. Every step is deterministic: min/max of
// FP32 values are exact and the sort is stable.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "internal.hpp"

namespace sonar {

namespace {

constexpr int BT = 256;                 // threads per block of the simple kernels
constexpr int RS_THREADS = 256;         // radix sort: threads per block
constexpr int RS_ITEMS = 8;             // radix sort: keys per thread per block
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int MAX_WALK = 4096;          // bound on parent-chain walks (a valid tree is far shallower)

// Order-preserving map of a float to a uint32 for atomic min/max.
__device__ __forceinline__ uint32_t f2ord(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// K1: bounds and centroids of every triangle; scene centroid box and vertex
// box via block reductions and ordered-int atomics. Validates indices and
// vertices.
__global__ void k_tri_prep(const float *__restrict__ V, int64_t nv, const int32_t *__restrict__ I,
                           const float *__restrict__ rho, const float *__restrict__ phi,
                           const uint8_t *__restrict__ mat, int64_t nt, float4 *__restrict__ tri_rec,
                           float4 *__restrict__ cen, float4 *__restrict__ blo, float4 *__restrict__ bhi,
                           uint32_t *__restrict__ part, int *__restrict__ status)
{
    __shared__ float s_min[6][BT / 64], s_max[6][BT / 64];
    int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    float mn[6], mx[6];
    for (int k = 0; k < 6; ++k) { mn[k] = INFINITY; mx[k] = -INFINITY; }
    if (i < nt) {
        int32_t a = I[3 * i], b = I[3 * i + 1], c = I[3 * i + 2];
        int bad = (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv);
        if (bad) {
            atomicOr(status, ST_BAD_INDEX);
            a = b = c = 0;
        }
        float v[9];
        for (int k = 0; k < 3; ++k) {
            v[k] = V[3 * (int64_t)a + k];
            v[3 + k] = V[3 * (int64_t)b + k];
            v[6 + k] = V[3 * (int64_t)c + k];
        }
        int nonfinite = 0;
        for (int k = 0; k < 9; ++k) nonfinite |= !isfinite(v[k]);
        float r = rho[i], p = phi[i];
        uint8_t m = mat[i];
        if (nonfinite || !isfinite(r) || !isfinite(p) || r < 0.f || m > 1) {
            atomicOr(status, ST_BAD_VERTEX);
            for (int k = 0; k < 9; ++k) v[k] = 0.f;
        }
        float3 lo = make_float3(fminf(v[0], fminf(v[3], v[6])), fminf(v[1], fminf(v[4], v[7])),
                                fminf(v[2], fminf(v[5], v[8])));
        float3 hi = make_float3(fmaxf(v[0], fmaxf(v[3], v[6])), fmaxf(v[1], fmaxf(v[4], v[7])),
                                fmaxf(v[2], fmaxf(v[5], v[8])));
        float3 cc = make_float3(0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z));
        uint32_t idbits = (uint32_t)i | (m ? MAT_BIT : 0u);
        tri_rec[3 * i + 0] = make_float4(v[0], v[1], v[2], v[3]);
        tri_rec[3 * i + 1] = make_float4(v[4], v[5], v[6], v[7]);
        tri_rec[3 * i + 2] = make_float4(v[8], __uint_as_float(idbits), r, p);
        cen[i] = make_float4(cc.x, cc.y, cc.z, 0.f);
        blo[i] = make_float4(lo.x, lo.y, lo.z, 0.f);
        bhi[i] = make_float4(hi.x, hi.y, hi.z, 0.f);
        mn[0] = cc.x; mn[1] = cc.y; mn[2] = cc.z; mx[0] = cc.x; mx[1] = cc.y; mx[2] = cc.z;
        mn[3] = lo.x; mn[4] = lo.y; mn[5] = lo.z; mx[3] = hi.x; mx[4] = hi.y; mx[5] = hi.z;
    }
    for (int k = 0; k < 6; ++k) {
        for (int off = 32; off > 0; off >>= 1) {
            mn[k] = fminf(mn[k], __shfl_xor(mn[k], off));
            mx[k] = fmaxf(mx[k], __shfl_xor(mx[k], off));
        }
    }
    int w = threadIdx.x / 64, l = threadIdx.x % 64;
    if (l == 0)
        for (int k = 0; k < 6; ++k) { s_min[k][w] = mn[k]; s_max[k][w] = mx[k]; }
    __syncthreads();
    if (threadIdx.x < 6) {
        int k = threadIdx.x;
        float a = INFINITY, b = -INFINITY;
        for (int q = 0; q < BT / 64; ++q) { a = fminf(a, s_min[k][q]); b = fmaxf(b, s_max[k][q]); }
        part[(int64_t)blockIdx.x * 12 + k] = f2ord(a);
        part[(int64_t)blockIdx.x * 12 + 6 + k] = f2ord(b);
    }
}

// Reductions of per-block partials by one block (no atomics on one address):
// twelve order-preserving min (0..5) / max (6..11) words, or one int maximum.
__global__ __launch_bounds__(1024) void k_reduce_bounds(const uint32_t *__restrict__ part, int nb,
                                                        uint32_t *__restrict__ red)
{
    __shared__ uint32_t s[12][16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t v[12];
    for (int k = 0; k < 12; ++k) v[k] = k < 6 ? 0xFFFFFFFFu : 0u;
    for (int b = t; b < nb; b += 1024)
        for (int k = 0; k < 12; ++k) {
            const uint32_t x = part[(int64_t)b * 12 + k];
            v[k] = k < 6 ? min(v[k], x) : max(v[k], x);
        }
    for (int k = 0; k < 12; ++k) {
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t o = __shfl_xor(v[k], off);
            v[k] = k < 6 ? min(v[k], o) : max(v[k], o);
        }
        if (lane == 0) s[k][w] = v[k];
    }
    __syncthreads();
    if (t < 12) {
        uint32_t r = t < 6 ? 0xFFFFFFFFu : 0u;
        for (int q = 0; q < 16; ++q) r = t < 6 ? min(r, s[t][q]) : max(r, s[t][q]);
        red[t] = r;
    }
}

__global__ __launch_bounds__(1024) void k_reduce_max(const int32_t *__restrict__ part, int nb, int32_t *__restrict__ out)
{
    __shared__ int32_t s[16];
    const int t = threadIdx.x;
    int32_t v = INT32_MIN;
    for (int b = t; b < nb; b += 1024) v = max(v, part[b]);
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    if ((t & 63) == 0) s[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
        int32_t r = INT32_MIN;
        for (int q = 0; q < 16; ++q) r = max(r, s[q]);
        *out = r;
    }
}

// Block maximum of one int per thread into part[blockIdx.x].
__device__ __forceinline__ void block_max_to(int v, int32_t *__restrict__ part)
{
    __shared__ int32_t s[BT / 64];
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = s[0];
        for (int q = 1; q < BT / 64; ++q) r = max(r, s[q]);
        part[blockIdx.x] = r;
    }
}

__device__ __forceinline__ uint64_t spread3_21(uint32_t x)
{
    uint64_t v = x & 0x1FFFFFu;
    v = (v | (v << 32)) & 0x1F00000000FFFFULL;
    v = (v | (v << 16)) & 0x1F0000FF0000FFULL;
    v = (v | (v << 8)) & 0x100F00F00F00F00FULL;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

// K2: 63-bit Morton code (21 bits per axis) of each centroid in the centroid box.
__global__ void k_morton(const float4 *__restrict__ cen, int64_t nt, const uint32_t *__restrict__ red,
                         uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= nt) return;
    float lo[3], ext[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = ord2f(red[k]);
        ext[k] = ord2f(red[6 + k]) - lo[k];
    }
    float4 c = cen[i];
    float cc[3] = {c.x, c.y, c.z};
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
        float t = ext[k] > 0.f ? (cc[k] - lo[k]) / ext[k] : 0.f;
        t = fminf(fmaxf(t, 0.f), 1.f);
        uint32_t v = (uint32_t)(t * 2097152.0f);
        q[k] = v > 2097151u ? 2097151u : v;
    }
    keys[i] = (spread3_21(q[0]) << 2) | (spread3_21(q[1]) << 1) | spread3_21(q[2]);
    vals[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (uint64 key, uint32 value), 8-bit digits.

__global__ void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n, int shift, uint32_t *__restrict__ hist,
                          int nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t i = base + r * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of n uint32 in place, in three launches over tiles of
// SCAN_TILE: tile sums, a scan of the tile sums, then each tile's scan with
// its offset. Loads and stores are coalesced; a tile is scanned in LDS.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 5); }    // LDS index with one pad word per 32

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(const uint32_t *__restrict__ a, int64_t n,
                                                            uint32_t *__restrict__ sums)
{
    __shared__ uint32_t ws[SCAN_THREADS / 64];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const int64_t i = base + r * SCAN_THREADS + t;
        s += i < n ? a[i] : 0u;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((t & 63) == 0) ws[t >> 6] = s;
    __syncthreads();
    if (t == 0) {
        uint32_t tot = 0;
        for (int q = 0; q < SCAN_THREADS / 64; ++q) tot += ws[q];
        sums[blockIdx.x] = tot;
    }
}

// Exclusive scan of the tile sums by one block, 1024 at a time with a carry.
__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *__restrict__ sums, int n)
{
    __shared__ uint32_t ws[16];
    __shared__ uint32_t carry;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) carry = 0u;
    __syncthreads();
    for (int b0 = 0; b0 < n; b0 += 1024) {
        const int i = b0 + t;
        const uint32_t v = i < n ? sums[i] : 0u;
        uint32_t x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(x, off);
            if (lane >= off) x += o;
        }
        if (lane == 63) ws[w] = x;
        __syncthreads();
        uint32_t add = carry;
        for (int q = 0; q < w; ++q) add += ws[q];
        if (i < n) sums[i] = add + x - v;
        __syncthreads();
        if (t == 1023) carry = add + x;
        __syncthreads();
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(uint32_t *__restrict__ a, int64_t n,
                                                            const uint32_t *__restrict__ sums)
{
    __shared__ uint32_t tile[SCAN_TILE + SCAN_TILE / 32];
    __shared__ uint32_t ws[SCAN_THREADS / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const int j = r * SCAN_THREADS + t;
        tile[scan_pad(j)] = base + j < n ? a[base + j] : 0u;
    }
    __syncthreads();
    // thread t scans its SCAN_ITEMS consecutive entries
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        v[q] = tile[scan_pad(t * SCAN_ITEMS + q)];
        s += v[q];
    }
    uint32_t x = s;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(x, off);
        if (lane >= off) x += o;
    }
    if (lane == 63) ws[w] = x;
    __syncthreads();
    uint32_t run = sums[blockIdx.x] + x - s;
    for (int q = 0; q < w; ++q) run += ws[q];
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        tile[scan_pad(t * SCAN_ITEMS + q)] = run;
        run += v[q];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const int j = r * SCAN_THREADS + t;
        if (base + j < n) a[base + j] = tile[scan_pad(j)];
    }
}

__global__ void k_rs_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, int64_t n,
                             int shift, const uint32_t *__restrict__ hist, int nblocks, uint64_t *__restrict__ kout,
                             uint32_t *__restrict__ vout)
{
    __shared__ uint32_t base[256], running[256], total[256];
    __shared__ uint32_t cnt[RS_WAVES][256];
    int t = threadIdx.x, w = t / 64, l = t % 64;
    base[t] = hist[(int64_t)t * nblocks + blockIdx.x];
    running[t] = 0;
    for (int q = 0; q < RS_WAVES; ++q) cnt[q][t] = 0;
    __syncthreads();
    const uint64_t lt_mask = (l == 0) ? 0ull : (~0ull >> (64 - l));
    int64_t tile = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t i = tile + r * RS_THREADS + t;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0ull;
        uint32_t val = valid ? vin[i] : 0u;
        uint32_t dig = (uint32_t)(key >> shift) & 0xFFu;
        uint64_t match = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            uint64_t bset = __ballot((dig >> bit) & 1u);
            match &= ((dig >> bit) & 1u) ? bset : ~bset;
        }
        uint32_t rank = __popcll(match & lt_mask);
        if (valid && rank == 0) cnt[w][dig] = __popcll(match);
        __syncthreads();
        {   // per-digit prefix over waves
            uint32_t p = 0;
            for (int q = 0; q < RS_WAVES; ++q) {
                uint32_t c = cnt[q][t];
                cnt[q][t] = p;
                p += c;
            }
            total[t] = p;
        }
        __syncthreads();
        if (valid) {
            uint32_t dst = base[dig] + running[dig] + cnt[w][dig] + rank;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        running[t] += total[t];
        for (int q = 0; q < RS_WAVES; ++q) cnt[q][t] = 0;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K4: binary radix tree over sorted keys. Internal node i covers a contiguous
// key range; equal keys are told apart by their index.

__device__ __forceinline__ int delta(const uint64_t *__restrict__ k, int64_t n, int64_t i, int64_t j)
{
    if (j < 0 || j >= n) return -1;
    uint64_t a = k[i], b = k[j];
    if (a != b) return __clzll(a ^ b);
    return 64 + __clz((uint32_t)(i ^ j));
}

__global__ void k_karras(const uint64_t *__restrict__ k, int64_t n, int32_t *__restrict__ left,
                         int32_t *__restrict__ right, int32_t *__restrict__ rlo, int32_t *__restrict__ rhi,
                         int32_t *__restrict__ parent)
{
    int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n - 1) return;
    int d = (delta(k, n, i, i + 1) - delta(k, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(k, n, i, i - d);
    int64_t lmax = 2;
    while (delta(k, n, i, i + lmax * d) > dmin) lmax *= 2;
    int64_t l = 0;
    for (int64_t t = lmax / 2; t >= 1; t /= 2)
        if (delta(k, n, i, i + (l + t) * d) > dmin) l += t;
    int64_t j = i + l * d;
    int dnode = delta(k, n, i, j);
    int64_t s = 0;
    int64_t t = l;
    do {
        t = (t + 1) / 2;
        if (delta(k, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int64_t gamma = i + s * d + (d < 0 ? d : 0);
    int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    // children: internal nodes 0..n-2, leaves encoded as n-1+leaf
    int32_t cl = (lo == gamma) ? (int32_t)(n - 1 + gamma) : (int32_t)gamma;
    int32_t cr = (hi == gamma + 1) ? (int32_t)(n - 1 + gamma + 1) : (int32_t)(gamma + 1);
    left[i] = cl;
    right[i] = cr;
    rlo[i] = (int32_t)lo;
    rhi[i] = (int32_t)hi;
    parent[cl] = (int32_t)i;
    parent[cr] = (int32_t)i;
}

// K5: bounds bottom-up, one tree level per launch. Every internal node's
// depth comes from walking its parent links (no dependence between threads);
// then the levels are merged from the deepest to the root, each launch
// reading only children finished by an earlier launch. Heights (edges to the
// deepest triangle) come along; the root's height is the hierarchy depth.
__global__ __launch_bounds__(BT) void k_depth(const int32_t *__restrict__ parent, int64_t n_int,
                                             int32_t *__restrict__ depth, int32_t *__restrict__ part,
                                             int *__restrict__ status)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    int d = 0;
    if (i < n_int) {
        int64_t p = i;
        while (p != 0 && d < MAX_WALK) {
            p = parent[p];
            ++d;
        }
        if (d >= MAX_WALK) atomicOr(status, ST_BAD_TREE);
        depth[i] = d;
    }
    block_max_to(d, part);
}

__global__ void k_leaf_boxes(const uint32_t *__restrict__ order, int64_t n, const float4 *__restrict__ blo_tri,
                             const float4 *__restrict__ bhi_tri, float4 *__restrict__ blo, float4 *__restrict__ bhi,
                             int32_t *__restrict__ height)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    const int64_t leaf = n - 1 + i;
    const uint32_t tri = order[i];
    blo[leaf] = blo_tri[tri];
    bhi[leaf] = bhi_tri[tri];
    height[leaf] = 0;
}

__global__ void k_refit_level(int level, int64_t n_int, const int32_t *__restrict__ depth,
                              const int32_t *__restrict__ left, const int32_t *__restrict__ right,
                              float4 *__restrict__ blo, float4 *__restrict__ bhi, int32_t *__restrict__ height)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n_int || depth[i] != level) return;
    const int32_t a = left[i], b = right[i];
    const float4 la = blo[a], ha = bhi[a];
    const float4 lb = blo[b], hb = bhi[b];
    blo[i] = make_float4(fminf(la.x, lb.x), fminf(la.y, lb.y), fminf(la.z, lb.z), 0.f);
    bhi[i] = make_float4(fmaxf(ha.x, hb.x), fmaxf(ha.y, hb.y), fmaxf(ha.z, hb.z), 0.f);
    height[i] = max(height[a], height[b]) + 1;
}

// K6: 4-wide nodes. A 4-wide node starts from a binary node's two children
// and opens, while it has fewer than four, the child of largest surface
// area that is not a leaf (a leaf: at most leaf_size consecutive triangle
// records), putting that child's two children in its place (the greedy
// collapse of a binary hierarchy by surface area, as wide-BVH builders do:
// large boxes, the ones rays most often enter, are split first). The
// children that are not leaves become 4-wide nodes in turn; the binary root
// is the top node. Which binary nodes become 4-wide nodes is decided top
// down, one binary depth per launch. Node layout, 8 float4: lo x, hi x, lo y,
// hi y, lo z, hi z of children 0..3, then the four child links; an empty
// child slot has an inverted box and the empty link.
__device__ __forceinline__ int32_t tri_count(int32_t c, int64_t n, const int32_t *rlo, const int32_t *rhi)
{
    return c >= n - 1 ? 1 : rhi[c] - rlo[c] + 1;
}

__device__ __forceinline__ float half_area(float4 l, float4 h)
{
    const float dx = h.x - l.x, dy = h.y - l.y, dz = h.z - l.z;
    return dx * dy + dy * dz + dz * dx;
}

// The children of the 4-wide node made from binary node x (2 to 4 of them).
__device__ int expand4(int32_t x, int64_t n, const int32_t *__restrict__ left, const int32_t *__restrict__ right,
                       const int32_t *__restrict__ rlo, const int32_t *__restrict__ rhi,
                       const float4 *__restrict__ blo, const float4 *__restrict__ bhi, int leaf_size, int32_t ch[4])
{
    int nc = 2;
    ch[0] = left[x];
    ch[1] = right[x];
    while (nc < 4) {
        int best = -1;
        float ba = -1.f;
        for (int q = 0; q < nc; ++q) {
            const int32_t c = ch[q];
            if (tri_count(c, n, rlo, rhi) <= leaf_size) continue;
            const float a = half_area(blo[c], bhi[c]);
            if (a > ba) {
                ba = a;
                best = q;
            }
        }
        if (best < 0) break;
        const int32_t c = ch[best];
        ch[best] = left[c];
        ch[nc++] = right[c];
    }
    return nc;
}

// The binary root becomes the top 4-wide node (level 0); no other node yet.
__global__ __launch_bounds__(BT) void k_mark4_root(int64_t n_int, uint32_t *__restrict__ flag,
                                                  int32_t *__restrict__ lev4)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n_int) return;
    flag[i] = i == 0 ? 1u : 0u;
    lev4[i] = 0;
}

// The 4-wide nodes of binary depth `level` (decided by their ancestors,
// which are shallower) mark their non-leaf children as 4-wide nodes one
// level further down.
__global__ __launch_bounds__(BT) void k_expand4(int level, int64_t n, const int32_t *__restrict__ depth,
                                               const int32_t *__restrict__ left, const int32_t *__restrict__ right,
                                               const int32_t *__restrict__ rlo, const int32_t *__restrict__ rhi,
                                               const float4 *__restrict__ blo, const float4 *__restrict__ bhi,
                                               int leaf_size, uint32_t *__restrict__ flag, int32_t *__restrict__ lev4)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n - 1 || depth[i] != level || !flag[i]) return;
    int32_t ch[4];
    const int nc = expand4((int32_t)i, n, left, right, rlo, rhi, blo, bhi, leaf_size, ch);
    for (int q = 0; q < nc; ++q) {
        const int32_t c = ch[q];
        if (tri_count(c, n, rlo, rhi) > leaf_size) {
            flag[c] = 1u;
            lev4[c] = lev4[i] + 1;
        }
    }
}

// Numbering input (the flags, scanned next) and the deepest 4-wide level.
__global__ __launch_bounds__(BT) void k_mark4(int64_t n_int, const uint32_t *__restrict__ flag,
                                             const int32_t *__restrict__ lev4, uint32_t *__restrict__ id4,
                                             int32_t *__restrict__ part)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    int lv = -1;
    if (i < n_int) {
        id4[i] = flag[i];
        if (flag[i]) lv = lev4[i];
    }
    block_max_to(lv, part);
}

__global__ void k_pack4(int64_t n, const int32_t *__restrict__ left, const int32_t *__restrict__ right,
                        const int32_t *__restrict__ rlo, const int32_t *__restrict__ rhi,
                        const float4 *__restrict__ blo, const float4 *__restrict__ bhi,
                        const uint32_t *__restrict__ flag, const uint32_t *__restrict__ id4, int leaf_size,
                        float4 *__restrict__ nodes)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n - 1 || !flag[i]) return;
    int32_t ch[4];
    const int nc = expand4((int32_t)i, n, left, right, rlo, rhi, blo, bhi, leaf_size, ch);
    float lo[3][4], hi[3][4];
    uint32_t link[4];
    for (int q = 0; q < 4; ++q) {
        if (q < nc) {
            const int32_t c = ch[q];
            const float4 l = blo[c], h = bhi[c];
            lo[0][q] = l.x; lo[1][q] = l.y; lo[2][q] = l.z;
            hi[0][q] = h.x; hi[1][q] = h.y; hi[2][q] = h.z;
            const int32_t cnt = tri_count(c, n, rlo, rhi);
            if (cnt <= leaf_size) {
                const uint32_t first = (uint32_t)(c >= n - 1 ? c - (n - 1) : rlo[c]);
                link[q] = LEAF_BIT | (first << 3) | (uint32_t)(cnt - 1);
            } else {
                link[q] = id4[c];
            }
        } else {
            for (int a = 0; a < 3; ++a) {
                lo[a][q] = INFINITY;
                hi[a][q] = -INFINITY;
            }
            link[q] = EMPTY_LINK;
        }
    }
    float4 *o = nodes + 8 * (size_t)id4[i];
    for (int a = 0; a < 3; ++a) {
        o[2 * a] = make_float4(lo[a][0], lo[a][1], lo[a][2], lo[a][3]);
        o[2 * a + 1] = make_float4(hi[a][0], hi[a][1], hi[a][2], hi[a][3]);
    }
    o[6] = make_float4(__uint_as_float(link[0]), __uint_as_float(link[1]), __uint_as_float(link[2]),
                       __uint_as_float(link[3]));
    o[7] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// A scene of at most leaf_size triangles: one node whose only child is a
// leaf over all of them.
__global__ void k_pack4_single(int64_t n, const float4 *__restrict__ tlo, const float4 *__restrict__ thi,
                               float4 *__restrict__ nodes)
{
    float l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t t = 0; t < n; ++t) {
        const float4 a = tlo[t], b = thi[t];
        l[0] = fminf(l[0], a.x); l[1] = fminf(l[1], a.y); l[2] = fminf(l[2], a.z);
        h[0] = fmaxf(h[0], b.x); h[1] = fmaxf(h[1], b.y); h[2] = fmaxf(h[2], b.z);
    }
    for (int a = 0; a < 3; ++a) {
        nodes[2 * a] = make_float4(l[a], INFINITY, INFINITY, INFINITY);
        nodes[2 * a + 1] = make_float4(h[a], -INFINITY, -INFINITY, -INFINITY);
    }
    nodes[6] = make_float4(__uint_as_float(LEAF_BIT | (uint32_t)(n - 1)), __uint_as_float(EMPTY_LINK),
                           __uint_as_float(EMPTY_LINK), __uint_as_float(EMPTY_LINK));
    nodes[7] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Checks every child link of the packed hierarchy: internal links inside the
// node array and not to the node itself, leaves inside the triangle array.
// Guards the traversal kernels against any malformed hierarchy.
__global__ void k_check_links4(const float4 *__restrict__ nodes, int64_t n_nodes, int64_t n_tri,
                               int *__restrict__ status)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n_nodes) return;
    const float4 d = nodes[8 * i + 6];
    const uint32_t l[4] = {__float_as_uint(d.x), __float_as_uint(d.y), __float_as_uint(d.z), __float_as_uint(d.w)};
    for (int c = 0; c < 4; ++c) {
        const uint32_t x = l[c];
        bool ok;
        if (x == EMPTY_LINK) ok = c > 0;
        else if (x & LEAF_BIT) ok = (int64_t)((x & 0x7FFFFFFFu) >> 3) + (int64_t)(x & 7u) + 1 <= n_tri;
        else ok = (int64_t)x < n_nodes && (int64_t)x != i;
        if (!ok) atomicOr(status, ST_BAD_TREE);
    }
}

__global__ void k_gather_tris(const uint32_t *__restrict__ order, int64_t n, const float4 *__restrict__ in,
                              float4 *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    uint32_t t = order[i];
    out[3 * i + 0] = in[3 * (int64_t)t + 0];
    out[3 * i + 1] = in[3 * (int64_t)t + 1];
    out[3 * i + 2] = in[3 * (int64_t)t + 2];
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + BT - 1) / BT); }
inline int64_t leaf_size_of(const sonar_mesh &m) { return m.leaf_size; }

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

#define BCHECK(x)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            snprintf(err, errlen, "%s: %s", #x, hipGetErrorString(e_));                 \
            return e_ == hipErrorOutOfMemory ? SONAR_E_NOMEM : SONAR_E_DEVICE;          \
        }                                                                                \
    } while (0)

sonar_status build_hierarchy(const sonar_mesh &m, hipStream_t s, Scene *out, char *err, size_t errlen)
{
    const int64_t n = m.n_triangles;
    const int64_t nv = m.n_vertices;
    // device copies of the inputs when they are host pointers
    DevBuf dV, dI, dR, dP, dM;
    const float *V = m.vertices;
    const int32_t *I = m.indices;
    const float *R = m.reflectivity;
    const float *P = m.phase;
    const uint8_t *M = m.material;
    if (!m.on_device) {
        BCHECK(hipMalloc(&dV.p, sizeof(float) * 3 * nv));
        BCHECK(hipMalloc(&dI.p, sizeof(int32_t) * 3 * n));
        BCHECK(hipMalloc(&dR.p, sizeof(float) * n));
        BCHECK(hipMalloc(&dP.p, sizeof(float) * n));
        BCHECK(hipMalloc(&dM.p, n));
        BCHECK(hipMemcpyAsync(dV.p, V, sizeof(float) * 3 * nv, hipMemcpyHostToDevice, s));
        BCHECK(hipMemcpyAsync(dI.p, I, sizeof(int32_t) * 3 * n, hipMemcpyHostToDevice, s));
        BCHECK(hipMemcpyAsync(dR.p, R, sizeof(float) * n, hipMemcpyHostToDevice, s));
        BCHECK(hipMemcpyAsync(dP.p, P, sizeof(float) * n, hipMemcpyHostToDevice, s));
        BCHECK(hipMemcpyAsync(dM.p, M, n, hipMemcpyHostToDevice, s));
        V = (const float *)dV.p;
        I = (const int32_t *)dI.p;
        R = (const float *)dR.p;
        P = (const float *)dP.p;
        M = (const uint8_t *)dM.p;
    }
    const int64_t n_int = n > 1 ? n - 1 : 1;
    const int64_t n_all = 2 * n - 1;
    DevBuf rec, cen, tlo, thi, red, k0, k1, v0, v1, hist, tsum, lft, rgt, rlo, rhi, par, blo, bhi, ndp, dep, hgt, bpart;
    int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
    BCHECK(hipMalloc(&rec.p, sizeof(float4) * 3 * n));
    BCHECK(hipMalloc(&cen.p, sizeof(float4) * n));
    BCHECK(hipMalloc(&tlo.p, sizeof(float4) * n));
    BCHECK(hipMalloc(&thi.p, sizeof(float4) * n));
    BCHECK(hipMalloc(&red.p, sizeof(uint32_t) * 12 + sizeof(int) * 2));
    BCHECK(hipMalloc(&k0.p, sizeof(uint64_t) * n));
    BCHECK(hipMalloc(&k1.p, sizeof(uint64_t) * n));
    BCHECK(hipMalloc(&v0.p, sizeof(uint32_t) * n));
    BCHECK(hipMalloc(&v1.p, sizeof(uint32_t) * n));
    BCHECK(hipMalloc(&hist.p, sizeof(uint32_t) * 256 * nblocks));
    const int64_t n_hist = (int64_t)256 * nblocks;
    const int n_scan = (int)((n_hist + SCAN_TILE - 1) / SCAN_TILE);
    BCHECK(hipMalloc(&tsum.p, sizeof(uint32_t) * n_scan));
    BCHECK(hipMalloc(&lft.p, sizeof(int32_t) * n_int));
    BCHECK(hipMalloc(&rgt.p, sizeof(int32_t) * n_int));
    BCHECK(hipMalloc(&rlo.p, sizeof(int32_t) * n_int));
    BCHECK(hipMalloc(&rhi.p, sizeof(int32_t) * n_int));
    BCHECK(hipMalloc(&par.p, sizeof(int32_t) * n_all));
    BCHECK(hipMalloc(&blo.p, sizeof(float4) * n_all));
    BCHECK(hipMalloc(&bhi.p, sizeof(float4) * n_all));
    BCHECK(hipMalloc(&ndp.p, sizeof(int32_t) * n_int));
    BCHECK(hipMalloc(&dep.p, sizeof(int32_t)));
    BCHECK(hipMalloc(&bpart.p, sizeof(uint32_t) * 12 * (size_t)nblk(n > n_int ? n : n_int)));
    BCHECK(hipMalloc(&hgt.p, sizeof(int32_t) * n_all));

    DevBuf flg, id4, lv4;
    BCHECK(hipMalloc(&flg.p, sizeof(uint32_t) * n_int));
    BCHECK(hipMalloc(&id4.p, sizeof(uint32_t) * n_int));
    BCHECK(hipMalloc(&lv4.p, sizeof(int32_t) * n_int));
    const int n_scan4 = (int)((n_int + SCAN_TILE - 1) / SCAN_TILE);
    DevBuf tsum4;
    BCHECK(hipMalloc(&tsum4.p, sizeof(uint32_t) * n_scan4));

    // scene-owned arrays (freed with the scene, also when the build fails)
    float4 *tris = nullptr;
    int *status = nullptr;
    if (hipMalloc(&tris, sizeof(float4) * 3 * n) != hipSuccess) {
        snprintf(err, errlen, "out of device memory for the scene");
        return SONAR_E_NOMEM;
    }
    out->tris = tris;
    if (hipMalloc(&status, sizeof(int)) != hipSuccess) {
        snprintf(err, errlen, "out of device memory for the scene");
        return SONAR_E_NOMEM;
    }
    out->status = status;

    uint32_t *redp = (uint32_t *)red.p;
    int *st_build = (int *)(redp + 12);
    BCHECK(hipMemsetAsync(status, 0, sizeof(int), s));
    BCHECK(hipMemsetAsync(st_build, 0, sizeof(int), s));
    BCHECK(hipMemsetAsync(par.p, 0, sizeof(int32_t) * n_all, s));
    k_tri_prep<<<nblk(n), BT, 0, s>>>(V, nv, I, R, P, M, n, (float4 *)rec.p, (float4 *)cen.p, (float4 *)tlo.p,
                                      (float4 *)thi.p, (uint32_t *)bpart.p, st_build);
    k_reduce_bounds<<<1, 1024, 0, s>>>((const uint32_t *)bpart.p, (int)nblk(n), redp);
    k_morton<<<nblk(n), BT, 0, s>>>((const float4 *)cen.p, n, redp, (uint64_t *)k0.p, (uint32_t *)v0.p);
    uint64_t *ka = (uint64_t *)k0.p, *kb = (uint64_t *)k1.p;
    uint32_t *va = (uint32_t *)v0.p, *vb = (uint32_t *)v1.p;
    for (int shift = 0; shift < 64; shift += 8) {
        k_rs_hist<<<nblocks, RS_THREADS, 0, s>>>(ka, n, shift, (uint32_t *)hist.p, nblocks);
        k_scan_tiles<<<n_scan, SCAN_THREADS, 0, s>>>((const uint32_t *)hist.p, n_hist, (uint32_t *)tsum.p);
        k_scan_sums<<<1, 1024, 0, s>>>((uint32_t *)tsum.p, n_scan);
        k_scan_apply<<<n_scan, SCAN_THREADS, 0, s>>>((uint32_t *)hist.p, n_hist, (const uint32_t *)tsum.p);
        k_rs_scatter<<<nblocks, RS_THREADS, 0, s>>>(ka, va, n, shift, (const uint32_t *)hist.p, nblocks, kb, vb);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    if (n > 1) {
        k_karras<<<nblk(n - 1), BT, 0, s>>>(ka, n, (int32_t *)lft.p, (int32_t *)rgt.p, (int32_t *)rlo.p,
                                            (int32_t *)rhi.p, (int32_t *)par.p);
    }
    k_leaf_boxes<<<nblk(n), BT, 0, s>>>(va, n, (const float4 *)tlo.p, (const float4 *)thi.p, (float4 *)blo.p,
                                        (float4 *)bhi.p, (int32_t *)hgt.p);
    int max_level = 0;
    if (n > 1) {
        // levels of the tree: one short synchronisation for the deepest level
        k_depth<<<nblk(n_int), BT, 0, s>>>((const int32_t *)par.p, n_int, (int32_t *)ndp.p, (int32_t *)bpart.p,
                                           st_build);
        k_reduce_max<<<1, 1024, 0, s>>>((const int32_t *)bpart.p, (int)nblk(n_int), (int32_t *)dep.p);
        BCHECK(hipMemcpyAsync(&max_level, dep.p, sizeof(int), hipMemcpyDeviceToHost, s));
        BCHECK(hipStreamSynchronize(s));
        if (max_level >= MAX_WALK) {
            snprintf(err, errlen, "internal error: malformed hierarchy");
            return SONAR_E_DEVICE;
        }
        for (int level = max_level; level >= 0; --level)
            k_refit_level<<<nblk(n_int), BT, 0, s>>>(level, n_int, (const int32_t *)ndp.p, (const int32_t *)lft.p,
                                                     (const int32_t *)rgt.p, (float4 *)blo.p, (float4 *)bhi.p,
                                                     (int32_t *)hgt.p);
    }
    // 4-wide nodes: mark top down (one launch per binary depth), number
    // (exclusive scan), count (a short synchronisation), pack
    int n4 = 0, levels4 = 1;
    if (n > leaf_size_of(m)) {
        k_mark4_root<<<nblk(n_int), BT, 0, s>>>(n_int, (uint32_t *)flg.p, (int32_t *)lv4.p);
        for (int level = 0; level <= max_level; ++level)
            k_expand4<<<nblk(n_int), BT, 0, s>>>(level, n, (const int32_t *)ndp.p, (const int32_t *)lft.p,
                                                 (const int32_t *)rgt.p, (const int32_t *)rlo.p,
                                                 (const int32_t *)rhi.p, (const float4 *)blo.p,
                                                 (const float4 *)bhi.p, m.leaf_size, (uint32_t *)flg.p,
                                                 (int32_t *)lv4.p);
        k_mark4<<<nblk(n_int), BT, 0, s>>>(n_int, (const uint32_t *)flg.p, (const int32_t *)lv4.p,
                                           (uint32_t *)id4.p, (int32_t *)bpart.p);
        k_reduce_max<<<1, 1024, 0, s>>>((const int32_t *)bpart.p, (int)nblk(n_int), (int32_t *)dep.p);
        k_scan_tiles<<<n_scan4, SCAN_THREADS, 0, s>>>((const uint32_t *)id4.p, n_int, (uint32_t *)tsum4.p);
        k_scan_sums<<<1, 1024, 0, s>>>((uint32_t *)tsum4.p, n_scan4);
        k_scan_apply<<<n_scan4, SCAN_THREADS, 0, s>>>((uint32_t *)id4.p, n_int, (const uint32_t *)tsum4.p);
        uint32_t last_id = 0, last_flag = 0;
        int max_lv = -1;
        BCHECK(hipMemcpyAsync(&last_id, (uint32_t *)id4.p + (n_int - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        BCHECK(hipMemcpyAsync(&last_flag, (uint32_t *)flg.p + (n_int - 1), sizeof(uint32_t), hipMemcpyDeviceToHost,
                              s));
        BCHECK(hipMemcpyAsync(&max_lv, dep.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BCHECK(hipStreamSynchronize(s));
        n4 = (int)(last_id + last_flag);
        levels4 = max_lv + 1;
    }
    const bool single = n4 == 0;
    if (single) n4 = 1;
    if (n4 > (1 << 25)) {      // traversal addresses nodes by 32-bit byte offsets
        snprintf(err, errlen, "hierarchy of %d nodes: at most 2^25 are supported", n4);
        return SONAR_E_UNSUPPORTED;
    }
    float4 *nodes = nullptr;
    if (hipMalloc(&nodes, sizeof(float4) * 8 * (size_t)n4) != hipSuccess) {
        snprintf(err, errlen, "out of device memory for the scene");
        return SONAR_E_NOMEM;
    }
    out->nodes = nodes;
    if (single) {
        k_pack4_single<<<1, 1, 0, s>>>(n, (const float4 *)tlo.p, (const float4 *)thi.p, nodes);
    } else {
        k_pack4<<<nblk(n - 1), BT, 0, s>>>(n, (const int32_t *)lft.p, (const int32_t *)rgt.p,
                                           (const int32_t *)rlo.p, (const int32_t *)rhi.p, (const float4 *)blo.p,
                                           (const float4 *)bhi.p, (const uint32_t *)flg.p, (const uint32_t *)id4.p,
                                           m.leaf_size, nodes);
    }
    k_gather_tris<<<nblk(n), BT, 0, s>>>(va, n, (const float4 *)rec.p, tris);
    k_check_links4<<<nblk(n4), BT, 0, s>>>(nodes, n4, n, st_build);
    BCHECK(hipGetLastError());
    uint32_t hred[12];
    int hst = 0, hdep = 0;
    BCHECK(hipMemcpyAsync(hred, redp, sizeof(hred), hipMemcpyDeviceToHost, s));
    BCHECK(hipMemcpyAsync(&hst, st_build, sizeof(int), hipMemcpyDeviceToHost, s));
    BCHECK(hipMemcpyAsync(&hdep, hgt.p, sizeof(int), hipMemcpyDeviceToHost, s));      // the binary root's height
    BCHECK(hipStreamSynchronize(s));
    if (hst & ST_BAD_INDEX) {
        snprintf(err, errlen, "triangle index outside [0, n_vertices)");
        return SONAR_E_INVALID;
    }
    if (hst & ST_BAD_TREE) {
        snprintf(err, errlen, "internal error: malformed hierarchy");
        return SONAR_E_DEVICE;
    }
    if (hst & ST_BAD_VERTEX) {
        snprintf(err, errlen, "non-finite vertex, reflectivity or phase, negative reflectivity or material > 1");
        return SONAR_E_INVALID;
    }
    auto ordf = [](uint32_t u) {
        uint32_t v = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
        float f;
        memcpy(&f, &v, 4);
        return f;
    };
    for (int k = 0; k < 3; ++k) {
        out->lo[k] = ordf(hred[3 + k]);
        out->hi[k] = ordf(hred[9 + k]);
    }
    out->zabs_max = fmaxf(fabsf(out->lo[2]), fabsf(out->hi[2]));
    out->n_tri = n;
    out->n_nodes = n4;
    out->depth = levels4;
    out->binary_depth = hdep;
    out->stack = 3 * levels4;     // a traversal pushes at most three children per level
    out->leaf_size = m.leaf_size;
    return SONAR_OK;
}

}  // namespace sonar
