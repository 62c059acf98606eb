// Learned multipath surrogate: kernels and host orchestration.
//
// Sec. II-B lets scattering and reverberation effects be learned from data.
// Here a small network maps each beam's single-bounce G-buffer (3 x 3 beam
// neighbourhood of 8 features: the first-hit statistics and the beam axis's
// vertical component) and the beam's geometry (mean first-hit point, beam
// axis, sensor position, the axis mirrored at the mean first-hit normal;
// sines and cosines of all but the sensor position at five octaves) to the
// first 64
// orthonormal DCT-II coefficients of the dB level, above the intensity
// floor, of what further bounces add to its range profile. Layers: 72
// im2col convolution columns + 102 geometry columns (174, zero-padded to
// 192) -> 64, then 64 -> 256 -> 256 -> 256 -> 64, ReLU between layers.
//
// Dense products run on the CDNA4 matrix cores: v_mfma_f32_16x16x32_bf16
// (BF16 operands, FP32 accumulation), 64 x 64 block tiles staged through LDS
// with k-contiguous fragments, three operand layouts (activations x W^T,
// dZ x W, X^T x dZ with a split reduction). Weights are FP32 master copies
// updated by Adam (Kingma and Ba, 2015) and mirrored in BF16 in the two
// layouts the products read. All reductions are two-stage in a fixed order,
// so a training step is bit-reproducible.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "internal.hpp"
#include "surrogate.hpp"

namespace sonar {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int NL = 5;                                       // layers
constexpr int NFEAT = 8;                                    // G-buffer features per beam
constexpr int NIM2COL = 9 * NFEAT;                          // 3 x 3 neighbourhood columns
constexpr int NGEO_FREQ = 5;                                // octaves of the geometry's sines and cosines
constexpr int NGEO = 12 + 18 * NGEO_FREQ;                   // geometry columns
constexpr int GEO_STRIDE = 16;                              // floats of one image's geometry block
constexpr int LK[NL] = {NIM2COL + NGEO, 64, 256, 256, 256}; // true fan-in
// padded fan-in: a multiple of 64, since the weight gradient X^T dZ has it as
// its row count and the products tile rows and columns by 64
constexpr int LKP[NL] = {(LK[0] + 63) / 64 * 64, 64, 256, 256, 256};
static_assert(LKP[0] % 64 == 0 && LKP[1] % 64 == 0 && LKP[2] % 64 == 0 && LKP[3] % 64 == 0 && LKP[4] % 64 == 0,
              "padded fan-ins tile by 64");
constexpr int LN[NL] = {64, 256, 256, 256, 64};             // fan-out
constexpr int NCOEF = 64;
constexpr int GB_STRIDE = 8;                                // floats per beam in the G-buffer
constexpr int TM = 64, TN = 64, TK = 32, LDT = TK + 8;      // GEMM tiles; LDS row stride in bf16
constexpr int SPLIT_ROWS = 4096;                            // reduction chunk of the weight gradients
constexpr float I_FLOOR = 1e-11f;

enum { EPI_BIAS_RELU = 0, EPI_BIAS = 1, EPI_MASK = 2, EPI_PARTIAL = 3 };

constexpr int64_t layer_param_offset(int l)
{
    int64_t o = 0;
    for (int i = 0; i < l; ++i) o += (int64_t)LK[i] * LN[i] + LN[i];
    return o;
}
constexpr int64_t N_PARAMS = layer_param_offset(NL);

// ---------------------------------------------------------------------------
// GEMM: C[M][N] = sum_k A(m, k) B(k, n), BF16 x BF16 -> FP32 on MFMA.
//   TA = false: A stored [M][K] (lda); TA = true: A stored [K][M] (lda).
//   TB = false: B stored [N][K] (ldb); TB = true: B stored [K][N] (ldb).
// M, N multiples of 64 and K a multiple of 32 (checked by the host). With
// split > 1, blockIdx.z reduces rows [z * kchunk, (z + 1) * kchunk) of K and
// writes FP32 partials [z][M][N].
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const __bf16 *__restrict__ A, int lda, const __bf16 *__restrict__ B,
                                              int ldb, int K, int kchunk, const float *__restrict__ bias,
                                              const __bf16 *__restrict__ mask, int ldm, void *__restrict__ out,
                                              int ldo, int M, int N)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[TM * LDT];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[TN * LDT];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kb; k0 < ke; k0 += TK) {
        // ---- stage A tile (64 rows x 32 k) as [m][k]
        if (!TA) {
            const int r = t >> 2, c = (t & 3) * 8;
            *reinterpret_cast<uint4 *>(&As[r * LDT + c]) =
                *reinterpret_cast<const uint4 *>(&A[(int64_t)(m0 + r) * lda + k0 + c]);
        } else {
            const int kk = t >> 3, c = (t & 7) * 8;
            uint4 v = *reinterpret_cast<const uint4 *>(&A[(int64_t)(k0 + kk) * lda + m0 + c]);
            const __bf16 *e = reinterpret_cast<const __bf16 *>(&v);
            for (int i = 0; i < 8; ++i) As[(c + i) * LDT + kk] = e[i];
        }
        // ---- stage B tile (32 k x 64 cols) as [n][k]
        if (!TB) {
            const int r = t >> 2, c = (t & 3) * 8;
            *reinterpret_cast<uint4 *>(&Bs[r * LDT + c]) =
                *reinterpret_cast<const uint4 *>(&B[(int64_t)(n0 + r) * ldb + k0 + c]);
        } else {
            const int kk = t >> 3, c = (t & 7) * 8;
            uint4 v = *reinterpret_cast<const uint4 *>(&B[(int64_t)(k0 + kk) * ldb + n0 + c]);
            const __bf16 *e = reinterpret_cast<const __bf16 *>(&v);
            for (int i = 0; i < 8; ++i) Bs[(c + i) * LDT + kk] = e[i];
        }
        __syncthreads();
        // ---- fragments: lane l holds row/col (l % 16), k = 8 (l / 16) .. + 7
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i)
            a[i] = *reinterpret_cast<const bf16x8 *>(&As[(wm + 16 * i + (lane & 15)) * LDT + 8 * (lane >> 4)]);
        for (int j = 0; j < 2; ++j)
            b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[(wn + 16 * j + (lane & 15)) * LDT + 8 * (lane >> 4)]);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // ---- epilogue: lane l holds column (l % 16), rows 4 (l / 16) .. + 3 of each 16 x 16 tile
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + e;
                const int n = n0 + wn + 16 * j + (lane & 15);
                float v = acc[i][j][e];
                if (EPI == EPI_BIAS_RELU) {
                    v += bias[n];
                    reinterpret_cast<__bf16 *>(out)[(int64_t)m * ldo + n] = (__bf16)(v > 0.f ? v : 0.f);
                } else if (EPI == EPI_BIAS) {
                    reinterpret_cast<float *>(out)[(int64_t)m * ldo + n] = v + bias[n];
                } else if (EPI == EPI_MASK) {
                    const float keep = (float)mask[(int64_t)m * ldm + n] > 0.f ? 1.f : 0.f;
                    reinterpret_cast<__bf16 *>(out)[(int64_t)m * ldo + n] = (__bf16)(v * keep);
                } else {
                    reinterpret_cast<float *>(out)[((int64_t)blockIdx.z * M + m) * ldo + n] = v;
                }
            }
}

// Geometry columns of beam (v, h) of a cell-centred H x W image, from the
// image's geometry block (sensor position, sensor-to-world rotation
// row-major, horizontal and vertical fields of view) and the beam's G-buffer
// entry: the beam axis u (world), the mean first hit P = S + r_max g0 u on it
// (the origin without a hit), the axis mirrored at the mean first-hit normal
// n (g3..g5), m = u - 2 (u . n) n / |n|^2 (zero without a hit or normal):
// where a specular continuation of the first hit heads. Columns: P / 10 (3),
// u (3), S / 10 (3), m (3), then sin(pi/2 2^k x), then cos(pi/2 2^k x), for
// x in (P / 10, u, m), x-major, k = 0 .. NGEO_FREQ - 1. Lengths in metres.
// Each column j goes out through put(j, value) as it is computed (no array
// of all columns held in registers).
template <class Put>
__device__ __forceinline__ void geo_columns(const float *__restrict__ geo, const float *__restrict__ gb, int v, int h,
                                            int H, int W, float r_max, Put put)
{
    const float hfov = geo[12], vfov = geo[13];
    const float az = -0.5f * hfov + ((float)h + 0.5f) * hfov / (float)W;
    const float el = -0.5f * vfov + ((float)v + 0.5f) * vfov / (float)H;
    float sa, ca, se, ce;
    sincosf(az, &sa, &ca);
    sincosf(el, &se, &ce);
    const float us0 = ce * ca, us1 = ce * sa, us2 = se;
    const bool hit = gb[6] > 0.f;
    const float r = r_max * gb[0];
    float x[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float u = geo[3 + 3 * i] * us0 + geo[4 + 3 * i] * us1 + geo[5 + 3 * i] * us2;
        x[3 + i] = u;
        x[i] = hit ? (geo[i] + r * u) * 0.1f : 0.f;
        put(6 + i, geo[i] * 0.1f);
    }
    const float nx = gb[3], ny = gb[4], nz = gb[5];
    const float nn = nx * nx + ny * ny + nz * nz;
    const bool mir = hit && nn > 1e-12f;
    const float f = mir ? 2.f * (x[3] * nx + x[4] * ny + x[5] * nz) / nn : 0.f;
    x[6] = mir ? x[3] - f * nx : 0.f;
    x[7] = mir ? x[4] - f * ny : 0.f;
    x[8] = mir ? x[5] - f * nz : 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) put(9 + i, x[6 + i]);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        if (q < 6) put(q, x[q]);
#pragma unroll
        for (int k = 0; k < NGEO_FREQ; ++k) {
            float sn, cs;
            sincosf(1.57079632679489662f * (float)(1 << k) * x[q], &sn, &cs);
            put(12 + q * NGEO_FREQ + k, sn);
            put(12 + 9 * NGEO_FREQ + q * NGEO_FREQ + k, cs);
        }
    }
}

// Geometry columns of the layer-0 input, and zeros in its padding columns,
// one thread per row.
__global__ void k_geo_cols(const float *__restrict__ g, const float *__restrict__ geo, int n_img, int H, int W,
                           float r_max, __bf16 *__restrict__ x)
{
    const int64_t rows = (int64_t)n_img * H * W;
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= rows) return;
    const int img = (int)(row / ((int64_t)H * W));
    const int rem = (int)(row % ((int64_t)H * W));
    __bf16 *xr = x + row * LKP[0] + NIM2COL;
    geo_columns(geo + (int64_t)img * GEO_STRIDE, g + row * GB_STRIDE, rem / W, rem % W, H, W, r_max,
                [&](int j, float v) { xr[j] = (__bf16)v; });
#pragma unroll
    for (int c = LK[0]; c < LKP[0]; ++c) x[row * LKP[0] + c] = (__bf16)0.f;
}

// im2col of the G-buffer: row (img, v, h) gets the 8 features of its 3 x 3
// neighbourhood ordered (dv, dh, feature), zero outside the image (k_geo_cols
// writes the remaining columns). One thread per (row, neighbour): two
// 16-byte loads and one 16-byte store.
__global__ void k_im2col(const float *__restrict__ g, int n_img, int H, int W, __bf16 *__restrict__ x)
{
    const int64_t rows = (int64_t)n_img * H * W;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * 9) return;
    const int64_t row = i / 9;
    const int q = (int)(i - row * 9);
    const int img = (int)(row / ((int64_t)H * W));
    const int rem = (int)(row - img * ((int64_t)H * W));
    const int vv = rem / W + q / 3 - 1, hh = rem % W + q % 3 - 1;
    float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
    if (vv >= 0 && vv < H && hh >= 0 && hh < W) {
        const float4 *src = reinterpret_cast<const float4 *>(g + (((int64_t)img * H + vv) * W + hh) * GB_STRIDE);
        lo = src[0];
        hi = src[1];
    }
    const bf16x8 w8 = {(__bf16)lo.x, (__bf16)lo.y, (__bf16)lo.z, (__bf16)lo.w,
                       (__bf16)hi.x, (__bf16)hi.y, (__bf16)hi.z, (__bf16)hi.w};
    *reinterpret_cast<bf16x8 *>(x + row * LKP[0] + q * NFEAT) = w8;      // rows of LKP[0] (a multiple of 64) bf16: aligned
}

// Weighted MSE on the 64 coefficients: dZ = 2 w_j (y - t) / (rows * 64) in
// BF16 and per block partial sums of w_j (y - t)^2 in FP64.
__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ t, const float *__restrict__ w,
                      int64_t n, __bf16 *__restrict__ dz, double *__restrict__ part)
{
    __shared__ double sh[256];
    const int64_t i0 = (int64_t)blockIdx.x * 256 * 16;
    double s = 0.0;
    const float sc = (float)(2.0 / (double)n);
    for (int q = 0; q < 16; ++q) {
        const int64_t i = i0 + (int64_t)q * 256 + threadIdx.x;
        if (i < n) {
            const float d = y[i] - t[i], wj = w[i & (NCOEF - 1)];
            dz[i] = (__bf16)(sc * wj * d);
            s += (double)wj * d * d;
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_loss_final(const double *__restrict__ part, int np, int64_t n, float *__restrict__ loss)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < np; ++i) s += part[i];
        *loss = (float)(s / (double)n);
    }
}

// Column sums of a BF16 [rows][N] matrix over row chunks of SPLIT_ROWS: FP32
// partials [chunk][N].
__global__ void k_colsum(const __bf16 *__restrict__ x, int64_t rows, int N, float *__restrict__ part)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r0 = (int64_t)blockIdx.x * SPLIT_ROWS;
    const int64_t r1 = min(rows, r0 + SPLIT_ROWS);
    __shared__ float sh[4][64];
    float s = 0.f;
    for (int64_t r = r0 + (threadIdx.x >> 6); r < r1; r += 4) s += (float)x[r * N + c];
    sh[threadIdx.x >> 6][threadIdx.x & 63] = s;
    __syncthreads();
    if (threadIdx.x < 64) part[(int64_t)blockIdx.x * N + c] = sh[0][threadIdx.x] + sh[1][threadIdx.x] +
                                                              sh[2][threadIdx.x] + sh[3][threadIdx.x];
}

// Sums split partials [S][K][N] (fixed order) into a flat parameter-gradient
// block: rows k < k_true go to grad[k * N + n] (the padded row is dropped).
__global__ void k_reduce_partials(const float *__restrict__ part, int S, int K, int N, int k_true,
                                  float *__restrict__ grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K * N) return;
    const int k = i / N;
    if (k >= k_true) return;
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += part[(int64_t)z * K * N + i];
    grad[i] = s;
}

// Adam on the flat FP32 master parameters (bias-corrected moments).
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 mirrors of layer l: wt [N][Kp] (k contiguous) and wk [Kp][N] (n
// contiguous), padded rows zero; FP32 bias copy.
__global__ void k_pack_layer(const float *__restrict__ master, int K, int Kp, int N, __bf16 *__restrict__ wt,
                             __bf16 *__restrict__ wk, float *__restrict__ bias)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < Kp * N) {
        const int k = i / N, n = i % N;
        const float v = k < K ? master[(int64_t)k * N + n] : 0.f;
        wt[(int64_t)n * Kp + k] = (__bf16)v;
        wk[(int64_t)k * N + n] = (__bf16)v;
    }
    if (i < N) bias[i] = master[(int64_t)K * N + i];
}

// Range smoothing of an incoherent channel: box average over bins
// [r - w/2, r + w/2), zero outside. One wave per row: the row is staged in
// LDS (one pad word per 16 so that the lanes' chunks spread over the banks),
// each lane slides an FP64 window sum over its consecutive bins, and the
// results leave through LDS with coalesced stores.
__device__ __forceinline__ int spad(int b) { return b + (b >> 4); }

__global__ __launch_bounds__(64) void k_smooth(const float *__restrict__ i1, const float *__restrict__ im, int nb,
                                               int w, float *__restrict__ s1, float *__restrict__ sm)
{
    extern __shared__ float lds[];     // input and output rows, padded
    const int lane = threadIdx.x;
    const int pitch = spad(nb) + 1;
    float *in = lds, *out = lds + pitch;
    const int64_t o = (int64_t)blockIdx.x * nb;
    const int per = (nb + 63) / 64;
    const int b0 = lane * per, b1 = min(b0 + per, nb);
    const double inv = 1.0 / w;
    for (int ch = i1 ? 0 : 1; ch < (im ? 2 : 1); ++ch) {
        const float *src = (ch ? im : i1) + o;
        float *dst = (ch ? sm : s1) + o;
#pragma unroll 8
        for (int b = lane; b < nb; b += 64) in[spad(b)] = src[b];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (b0 < nb) {
            double acc = 0.0;
            for (int q = max(0, b0 - w / 2); q < min(nb, b0 + w - w / 2); ++q) acc += (double)in[spad(q)];
            out[spad(b0)] = (float)(acc * inv);
            for (int b = b0 + 1; b < b1; ++b) {
                const int enter = b + w - w / 2 - 1, leave = b - w / 2 - 1;
                if (enter < nb) acc += (double)in[spad(enter)];
                if (leave >= 0) acc -= (double)in[spad(leave)];
                out[spad(b)] = (float)(acc * inv);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 8
        for (int b = lane; b < nb; b += 64) __builtin_nontemporal_store(out[spad(b)], dst + b);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Bin of a beam's mean first-bounce range from its G-buffer (feature 0 is
// range / r_max, feature 6 the hit fraction); 0 when it has no hits.
__device__ __forceinline__ int first_hit_bin(const float *__restrict__ g, int64_t row, float r_min, float r_max,
                                             float dr, int nb)
{
    const float f0 = g[row * GB_STRIDE + 0], cnt = g[row * GB_STRIDE + 6];
    if (!(cnt > 0.f)) return 0;
    const float b = floorf((f0 * r_max - r_min) / dr);
    return (int)fminf(fmaxf(b, 0.f), (float)(nb - 1));
}

// Level target: for each row, c_j = sum_r' C[j][r'] lev[r' + r1], with
// lev = 10 log10(1 + Ims / floor) the dB level of the range-smoothed
// later-bounce channel above the floor, shifted so the beam's first-hit bin
// r1 is bin 0 (zero past the end), optionally standardised
// (c - mu_j) / sigma_j. Block: 64 rows x 64 coefficients; bins staged 64 at a
// time in LDS.
__global__ __launch_bounds__(256) void k_level_coef(const float *__restrict__ im, const float *__restrict__ gbuf,
                                                    int64_t rows, int nb, float r_min, float r_max,
                                                    const float *__restrict__ basis, const float *__restrict__ mu,
                                                    const float *__restrict__ sg, int standardize,
                                                    float *__restrict__ coef)
{
    __shared__ float R[64][65];
    __shared__ float Cb[64][65];
    __shared__ int r1s[64];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const float dr = (r_max - r_min) / nb;
    if (t < 64) r1s[t] = (r0 + t < rows) ? first_hit_bin(gbuf, r0 + t, r_min, r_max, dr, nb) : 0;
    __syncthreads();
    const int rr = t >> 2;           // row within the block handled by this thread
    const int cq = (t & 3) * 16;     // first of its 16 coefficients
    float acc[16];
    for (int q = 0; q < 16; ++q) acc[q] = 0.f;
    for (int b0 = 0; b0 < nb; b0 += 64) {
        for (int e = t; e < 64 * 64; e += 256) {
            const int r = e >> 6, b = e & 63;
            float v = 0.f;
            const int src = b0 + b + r1s[r];
            if (r0 + r < rows && src < nb) v = 10.f * log10f(1.f + im[(r0 + r) * nb + src] * (1.f / I_FLOOR));
            R[r][b] = v;
            Cb[r][b] = (b0 + b < nb) ? basis[(int64_t)r * nb + b0 + b] : 0.f;
        }
        __syncthreads();
        for (int b = 0; b < 64; ++b) {
            const float x = R[rr][b];
            for (int q = 0; q < 16; ++q) acc[q] += Cb[cq + q][b] * x;
        }
        __syncthreads();
    }
    if (r0 + rr < rows) {
        for (int q = 0; q < 16; ++q) {
            const int j = cq + q;
            float v = acc[q];
            if (standardize) v = (v - mu[j]) / sg[j];
            coef[(r0 + rr) * NCOEF + j] = v;
        }
    }
}

// Column sums of v and v^2 of an FP32 [rows][64] matrix in FP64 partials.
__global__ void k_coef_moments(const float *__restrict__ c, int64_t rows, double *__restrict__ part)
{
    const int j = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * SPLIT_ROWS, r1 = min(rows, r0 + SPLIT_ROWS);
    __shared__ double s1[4][64], s2[4][64];
    double a = 0.0, b = 0.0;
    for (int64_t r = r0 + q; r < r1; r += 4) {
        const double v = c[r * NCOEF + j];
        a += v;
        b += v * v;
    }
    s1[q][j] = a;
    s2[q][j] = b;
    __syncthreads();
    if (q == 0) {
        part[(int64_t)blockIdx.x * 128 + j] = s1[0][j] + s1[1][j] + s1[2][j] + s1[3][j];
        part[(int64_t)blockIdx.x * 128 + 64 + j] = s2[0][j] + s2[1][j] + s2[2][j] + s2[3][j];
    }
}

// Mean level per bin: the inverse DCT of the mean coefficients (for the
// mean-level baseline error).
__global__ void k_mean_level(const float *__restrict__ basis, const float *__restrict__ mu, int nb,
                                float *__restrict__ mres)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    float a = 0.f;
    for (int j = 0; j < NCOEF; ++j) a += basis[(int64_t)j * nb + c] * mu[j];
    mres[c] = a;
}

// Predicted profile and per-beam dB errors. For row k with first-hit bin
// r1: profile[b] = 10 log10(I1[b] + floor 10^(lev[b] / 10)) at full range
// resolution, lev[b] = Q[k][b - r1] from r1 on and 0 before it, with
// Q[k][c] = sum_j C[j][c] c_kj the inverse DCT of the de-standardised
// prediction (a zero level leaves the single-bounce profile). Errors, as
// mean |error| in dB per beam:
//  the range-smoothed prediction 10 log10(I1s + floor 10^(lev / 10)) over
//  bins whose smoothed truth 10 log10(I1s + Ims + floor) is more than 3 dB
//  above the floor: [0] the prediction, [1] the smoothed single bounce,
//  [2] the smoothed single bounce plus the mean level, [3] the bin count;
//  the full-resolution profile over bins whose raw truth
//  10 log10(I1 + Im + floor) is more than 3 dB above the floor: [4] the
//  prediction, [5] the single bounce plus the mean level, [6] the single
//  bounce 10 log10(I1 + floor), [7] the bin count.
// Block: 16 rows, 4 waves, in two phases.
//  1. Q on the matrix cores, wave q taking a quarter of the columns c: 16 x
//     16 x 4 FP32 MFMA steps, A the 16 rows' coefficients (lane l: row l % 16,
//     coefficient 4 s + l / 16, in registers), B the basis (lane l:
//     coefficient 4 s + l / 16, column l % 16, generated in registers by a
//     cosine recurrence); lane l ends with Q of rows 4 (l / 16) + i, column
//     l % 16, stored to LDS.
//  2. The rows stream out, each thread taking bins t, t + 256, ... (P of
//     them); the single-bounce values of all 16 rows are loaded before phase
//     1, so their latency hides behind the matrix work. Error sums: wave
//     shuffles, then one LDS slot per wave and row.
constexpr int PR_ROWS = 16;

// 10 log10(x) from the hardware base-2 logarithm (about one ulp for the
// normal, positive arguments here: x >= the 1e-11 floor).
__device__ __forceinline__ float db10(float x) { return 3.01029995663981195f * __log2f(x); }

constexpr int N_ERR = 8;
constexpr float DB_TO_LOG2 = 0.332192809488736235f;     // log2(10) / 10

template <int P>
__global__ __launch_bounds__(256) void k_profile_errors(const float *__restrict__ pred, const float *__restrict__ i1r,
                                                        const float *__restrict__ imr, const float *__restrict__ i1s,
                                                        const float *__restrict__ ims, const float *__restrict__ gbuf,
                                                        int64_t rows, int nb, float r_min, float r_max,
                                                        const float *__restrict__ mu, const float *__restrict__ sg,
                                                        const float *__restrict__ mlev, float *__restrict__ err,
                                                        float *__restrict__ profile)
{
    extern __shared__ float Q[];              // [PR_ROWS][nb + 1]
    __shared__ int r1s[PR_ROWS];
    __shared__ float red[PR_ROWS][4][N_ERR];
    const int t = threadIdx.x, lane = t & 63, wq = t >> 6;
    const int ar = lane & 15, kq = lane >> 4;
    const int pitch = nb + 1;
    const int64_t r0 = (int64_t)blockIdx.x * PR_ROWS;
    const float dr = (r_max - r_min) / nb;
    const float occ_db = db10(I_FLOOR) + 3.f;
    if (t < PR_ROWS) r1s[t] = (r0 + t < rows) ? first_hit_bin(gbuf, r0 + t, r_min, r_max, dr, nb) : nb;
    // the raw single-bounce channel of the 16 rows, in flight during phase 1
    float iv[PR_ROWS][P];
#pragma unroll
    for (int rl = 0; rl < PR_ROWS; ++rl) {
        const int64_t rowc = min(r0 + rl, rows - 1);
#pragma unroll
        for (int q = 0; q < P; ++q) iv[rl][q] = i1r[rowc * nb + min(t + 256 * q, nb - 1)];
    }

    // phase 1: Q of this wave's column quarter
    float a[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int j = 4 * s + kq;
        a[s] = (r0 + ar < rows) ? pred[(r0 + ar) * NCOEF + j] * sg[j] + mu[j] : 0.f;
    }
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int cq = (nb + 3) / 4;
    const int c_begin = wq * cq, c_end = min(nb, c_begin + cq);
    // Basis values in registers: C[j][c] = s_j cos(j x_c), x_c = pi (c + 1/2) / nb.
    // This lane needs j = kq + 4 s at column c: seeds cos(kq x) and cos((kq + 4) x),
    // then cos((m + 1) 4x + kq x) = 2 cos(4x) cos(m 4x + kq x) - cos((m - 1) 4x + kq x).
    // The seeds and 4x advance by 16 columns per tile through exact rotations.
    const float dxc = 3.14159265358979323846f / nb;
    const float xa = (c_begin + ar + 0.5f) * dxc;
    float ca, sa, cb, sb, c4, s4, rca, rsa, rcb, rsb, rc4, rs4;
    sincosf(kq * xa, &sa, &ca);
    sincosf((kq + 4) * xa, &sb, &cb);
    sincosf(4.f * xa, &s4, &c4);
    sincosf(16.f * kq * dxc, &rsa, &rca);
    sincosf(16.f * (kq + 4) * dxc, &rsb, &rcb);
    sincosf(64.f * dxc, &rs4, &rc4);
    const float s0 = sqrtf(1.f / nb), s1 = sqrtf(2.f / nb);
    for (int c0 = c_begin; c0 < c_end; c0 += 16) {
        const int cc = c0 + ar;
        float bv[16];
        {
            const float r = 2.f * c4;
            float cm2 = ca, cm1 = cb;
            bv[0] = ca * (kq == 0 ? s0 : s1);
            bv[1] = cb * s1;
#pragma unroll
            for (int s = 2; s < 16; ++s) {
                const float cn = r * cm1 - cm2;
                bv[s] = cn * s1;
                cm2 = cm1;
                cm1 = cn;
            }
        }
        f4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 16; ++s) d = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bv[s], d, 0, 0, 0);
        {   // next tile: rotate the seeds by 16 columns
            float t = ca * rca - sa * rsa;
            sa = sa * rca + ca * rsa;
            ca = t;
            t = cb * rcb - sb * rsb;
            sb = sb * rcb + cb * rsb;
            cb = t;
            t = c4 * rc4 - s4 * rs4;
            s4 = s4 * rc4 + c4 * rs4;
            c4 = t;
        }
        if (cc < c_end) {
#pragma unroll
            for (int i = 0; i < 4; ++i) Q[(4 * kq + i) * pitch + cc] = d[i];
        }
    }
    __syncthreads();

    // phase 2: stream the rows out
#pragma unroll
    for (int rp = 0; rp < PR_ROWS; rp += 2) {
        float mv[2][P];
        if (imr) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t rowc = min(r0 + rp + h, rows - 1);
#pragma unroll
                for (int q = 0; q < P; ++q) mv[h][q] = imr[rowc * nb + min(t + 256 * q, nb - 1)];
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int rl = rp + h;
            const int64_t row = r0 + rl;
            const bool rok = row < rows;
            const int r1 = r1s[rl];
            float e[N_ERR];
#pragma unroll
            for (int k = 0; k < N_ERR; ++k) e[k] = 0.f;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int b = t + 256 * q;
                if (!rok || b >= nb) continue;
                const float ar = iv[rl][q];
                const float lev = b >= r1 ? Q[rl * pitch + (b - r1)] : 0.f;
                const float fl = I_FLOOR * exp2f(lev * DB_TO_LOG2);     // floor + predicted later-bounce intensity
                const float ph = db10(ar + fl);
                if (profile) __builtin_nontemporal_store(ph, profile + row * nb + b);      // streamed out
                if (imr) {
                    const float fm = I_FLOOR * exp2f(((b >= r1 && mlev) ? mlev[b - r1] : 0.f) * DB_TO_LOG2);
                    const float as = i1s[row * nb + b];
                    const float ts = db10(as + ims[row * nb + b] + I_FLOOR);
                    if (ts > occ_db) {
                        e[0] += fabsf(db10(as + fl) - ts);
                        e[1] += fabsf(db10(as + I_FLOOR) - ts);
                        e[2] += fabsf(db10(as + fm) - ts);
                        e[3] += 1.f;
                    }
                    const float tr = db10(ar + mv[h][q] + I_FLOOR);
                    if (tr > occ_db) {
                        e[4] += fabsf(ph - tr);
                        e[5] += fabsf(db10(ar + fm) - tr);
                        e[6] += fabsf(db10(ar + I_FLOOR) - tr);
                        e[7] += 1.f;
                    }
                }
            }
            if (err) {
#pragma unroll
                for (int k = 0; k < N_ERR; ++k)
                    for (int off = 32; off > 0; off >>= 1) e[k] += __shfl_xor(e[k], off);
                if (lane == 0) {
#pragma unroll
                    for (int k = 0; k < N_ERR; ++k) red[rl][wq][k] = e[k];
                }
            }
        }
    }
    if (!err) return;
    __syncthreads();
    if (t < PR_ROWS && r0 + t < rows) {
        float sm[N_ERR];
        for (int q = 0; q < N_ERR; ++q) sm[q] = red[t][0][q] + red[t][1][q] + red[t][2][q] + red[t][3][q];
        float *o = err + (r0 + t) * N_ERR;
        for (int g = 0; g < 2; ++g) {
            const float n = sm[4 * g + 3];
            for (int q = 0; q < 3; ++q) o[4 * g + q] = n > 0.f ? sm[4 * g + q] / n : NAN;
            o[4 * g + 3] = n;
        }
    }
}

// ---------------------------------------------------------------------------
// Fused inference: all five layers for a tile of MLP_ROWS rows in one block.
// The tile's activations stay in LDS (BF16, one buffer the layers overwrite
// in place: every wave finishes reading a layer's input before any writes
// its output), the accumulators in registers. Wave w owns a quarter of each
// layer's output columns for all MLP_ROWS rows; its weight fragments come
// straight from the k-contiguous BF16 mirror wt[l] [N][Kp] (L2-resident,
// each fragment read by one wave of the block), loaded one k-step ahead of
// the products that use them. Products, bias, ReLU and BF16 rounding are
// those of the layer-by-layer path, in the same k order.
constexpr int MLP_ROWS = 64;
constexpr int MLP_LDA = 256 + 8;          // LDS row pitch in bf16 (16 B pad against bank conflicts)
constexpr int L0_K = (LK[0] + 31) / 32 * 32;   // layer-0 fan-in rounded up to the k-step (32)
static_assert(L0_K <= LKP[0] && L0_K + 8 <= MLP_LDA, "layer-0 input fits the padded weights and the LDS row");

struct MlpWeights {
    const __bf16 *wt[NL];
    const float *bias[NL];
};

template <int K, int N>
__device__ __forceinline__ void mlp_layer(const __bf16 *__restrict__ act, const __bf16 *__restrict__ wt, int ldw,
                                          int wave, int lane, f32x4 (&acc)[4][N / 64])
{
    constexpr int NT = N / 64;            // 16-column tiles per wave
    const int ncol0 = wave * (N / 4);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 b[NT], bn[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j)
        b[j] = *reinterpret_cast<const bf16x8 *>(wt + (int64_t)(ncol0 + 16 * j + (lane & 15)) * ldw + 8 * (lane >> 4));
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 32) {
        if (k0 + 32 < K) {
#pragma unroll
            for (int j = 0; j < NT; ++j)
                bn[j] = *reinterpret_cast<const bf16x8 *>(wt + (int64_t)(ncol0 + 16 * j + (lane & 15)) * ldw + k0 +
                                                          32 + 8 * (lane >> 4));
        }
        bf16x8 a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a[i] = *reinterpret_cast<const bf16x8 *>(act + (16 * i + (lane & 15)) * MLP_LDA + k0 + 8 * (lane >> 4));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (k0 + 32 < K) {
#pragma unroll
            for (int j = 0; j < NT; ++j) b[j] = bn[j];
        }
    }
}

// bias + ReLU + BF16 into the activation tile (after the barrier that ends
// every wave's reads of the layer input)
template <int N>
__device__ __forceinline__ void mlp_store(__bf16 *__restrict__ act, const float *__restrict__ bias, int wave, int lane,
                                          const f32x4 (&acc)[4][N / 64])
{
    constexpr int NT = N / 64;
    const int ncol0 = wave * (N / 4);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int n = ncol0 + 16 * j + (lane & 15);
        const float bn = bias[n];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float v = acc[i][j][e] + bn;
                act[(16 * i + 4 * (lane >> 4) + e) * MLP_LDA + n] = (__bf16)(v > 0.f ? v : 0.f);
            }
    }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ g, const float *__restrict__ geo,
                                                     int H, int W, float r_max, MlpWeights wts, float *__restrict__ y)
{
    __shared__ __attribute__((aligned(16))) __bf16 act[MLP_ROWS * MLP_LDA];
    __shared__ int rpos[MLP_ROWS][3];     // image, v, h of each row
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * MLP_ROWS;
    const int64_t hw = (int64_t)H * W;
    // layer-0 input. Each row's image and beam are decoded once (the 64-bit
    // and run-time divisions stay out of the per-element loop); its geometry
    // columns come from one thread per row
    if (t < MLP_ROWS) {
        const int64_t row = r0 + t;
        const int img = (int)(row / hw);
        const int rem = (int)(row - img * hw);
        const int v = rem / W, h = rem - (rem / W) * W;
        rpos[t][0] = img;
        rpos[t][1] = v;
        rpos[t][2] = h;
        __bf16 *ar = act + t * MLP_LDA + NIM2COL;
        geo_columns(geo + (int64_t)img * GEO_STRIDE, g + row * GB_STRIDE, v, h, H, W, r_max,
                    [&](int j, float val) { ar[j] = (__bf16)val; });
#pragma unroll
        for (int c = LK[0]; c < L0_K; ++c) act[t * MLP_LDA + c] = (__bf16)0.f;
    }
    __syncthreads();
    // the 3 x 3 neighbourhood features, one (row, neighbour) pair per step:
    // its 8 G-buffer floats as two 16-byte loads (zero outside the image)
    // and one 16-byte LDS store
    for (int e = t; e < MLP_ROWS * 9; e += 256) {
        const int r = e / 9, q = e - (e / 9) * 9;
        const int vv = rpos[r][1] + q / 3 - 1, hh = rpos[r][2] + q % 3 - 1;
        float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
        if (vv >= 0 && vv < H && hh >= 0 && hh < W) {
            const float4 *src = reinterpret_cast<const float4 *>(
                g + (((int64_t)rpos[r][0] * H + vv) * W + hh) * GB_STRIDE);
            lo = src[0];
            hi = src[1];
        }
        const bf16x8 w8 = {(__bf16)lo.x, (__bf16)lo.y, (__bf16)lo.z, (__bf16)lo.w,
                           (__bf16)hi.x, (__bf16)hi.y, (__bf16)hi.z, (__bf16)hi.w};
        *reinterpret_cast<bf16x8 *>(act + r * MLP_LDA + q * NFEAT) = w8;      // 16-byte aligned
    }
    __syncthreads();
    {
        f32x4 acc[4][1];
        mlp_layer<L0_K, 64>(act, wts.wt[0], LKP[0], wave, lane, acc);
        __syncthreads();
        mlp_store<64>(act, wts.bias[0], wave, lane, acc);
        __syncthreads();
    }
    {
        f32x4 acc[4][4];
        mlp_layer<64, 256>(act, wts.wt[1], LKP[1], wave, lane, acc);
        __syncthreads();
        mlp_store<256>(act, wts.bias[1], wave, lane, acc);
        __syncthreads();
    }
    for (int l = 2; l <= 3; ++l) {
        f32x4 acc[4][4];
        mlp_layer<256, 256>(act, wts.wt[l], LKP[l], wave, lane, acc);
        __syncthreads();
        mlp_store<256>(act, wts.bias[l], wave, lane, acc);
        __syncthreads();
    }
    {
        f32x4 acc[4][1];
        mlp_layer<256, 64>(act, wts.wt[4], LKP[4], wave, lane, acc);
        const int n = wave * 16 + (lane & 15);
        const float bn = wts.bias[4][n];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                y[(r0 + 16 * i + 4 * (lane >> 4) + e) * NCOEF + n] = acc[i][0][e] + bn;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side

struct Surrogate {
    int64_t max_rows = 0;
    int n_bins = 0;
    float *master = nullptr, *adam_m = nullptr, *adam_v = nullptr, *grad = nullptr;
    __bf16 *wt[NL] = {}, *wk[NL] = {};
    float *bias[NL] = {};
    __bf16 *x[NL] = {};          // layer inputs x0 .. x4
    __bf16 *dz[2] = {};          // ping-pong gradient buffers [rows][256]
    float *y = nullptr;          // [rows][64]
    float *part = nullptr;       // split partials [S][256][256]
    double *dpart = nullptr;     // loss / moment partials
    float *basis = nullptr;      // [64][n_bins]
    float *s1 = nullptr, *sm = nullptr;   // range-smoothed channels [max_rows][n_bins]
    float *mlev = nullptr;                // mean-level profile [n_bins]
    float *lw = nullptr;                  // loss weights [64]
    float r_min = 0.f, r_max = 0.f;
    int smooth = 32;
    float *mu = nullptr, *sg = nullptr;
    int64_t step = 0;
    std::vector<void *> allocs;
};

static hipError_t salloc(Surrogate *s, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) s->allocs.push_back(*p);
    return e;
}

void surrogate_free(Surrogate *s)
{
    if (!s) return;
    for (void *p : s->allocs) (void)hipFree(p);
    delete s;
}

int64_t surrogate_param_count() { return N_PARAMS; }

hipError_t surrogate_create(int64_t max_rows, int n_bins, float r_min, float r_max, int smooth, Surrogate **out)
{
    Surrogate *s = new (std::nothrow) Surrogate();
    if (!s) return hipErrorOutOfMemory;
    s->max_rows = max_rows;
    s->n_bins = n_bins;
    s->r_min = r_min;
    s->r_max = r_max;
    s->smooth = smooth;
    hipError_t e = hipSuccess;
#define SA(ptr, bytes)                                                        \
    do {                                                                      \
        if (e == hipSuccess) e = salloc(s, (void **)&(ptr), (size_t)(bytes)); \
    } while (0)
    SA(s->master, N_PARAMS * 4);
    SA(s->adam_m, N_PARAMS * 4);
    SA(s->adam_v, N_PARAMS * 4);
    SA(s->grad, N_PARAMS * 4);
    for (int l = 0; l < NL; ++l) {
        SA(s->wt[l], (size_t)LKP[l] * LN[l] * 2);
        SA(s->wk[l], (size_t)LKP[l] * LN[l] * 2);
        SA(s->bias[l], (size_t)LN[l] * 4);
        SA(s->x[l], (size_t)max_rows * LKP[l] * 2);
    }
    SA(s->dz[0], (size_t)max_rows * 256 * 2);
    SA(s->dz[1], (size_t)max_rows * 256 * 2);
    SA(s->y, (size_t)max_rows * NCOEF * 4);
    const int64_t S = (max_rows + SPLIT_ROWS - 1) / SPLIT_ROWS;
    SA(s->part, (size_t)S * 256 * 256 * 4);
    SA(s->dpart, (size_t)(max_rows / 4096 + S + 2) * 128 * 8);
    SA(s->basis, (size_t)NCOEF * n_bins * 4);
    SA(s->s1, (size_t)max_rows * n_bins * 4);
    SA(s->sm, (size_t)max_rows * n_bins * 4);
    SA(s->mlev, (size_t)n_bins * 4);
    SA(s->lw, NCOEF * 4);
    SA(s->mu, NCOEF * 4);
    SA(s->sg, NCOEF * 4);
#undef SA
    if (e != hipSuccess) {
        surrogate_free(s);
        return e;
    }
    // orthonormal DCT-II basis, first 64 rows, computed in FP64 on the host
    std::vector<float> B((size_t)NCOEF * n_bins);
    for (int j = 0; j < NCOEF; ++j)
        for (int r = 0; r < n_bins; ++r) {
            double sc = j == 0 ? sqrt(1.0 / n_bins) : sqrt(2.0 / n_bins);
            B[(size_t)j * n_bins + r] = (float)(sc * cos(M_PI * (r + 0.5) * j / n_bins));
        }
    std::vector<float> mu(NCOEF, 0.f), sg(NCOEF, 1.f), zero(N_PARAMS, 0.f);
    e = hipMemcpy(s->basis, B.data(), B.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->mu, mu.data(), NCOEF * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->sg, sg.data(), NCOEF * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->lw, sg.data(), NCOEF * 4, hipMemcpyHostToDevice);   // weights 1
    for (float **p : {&s->master, &s->adam_m, &s->adam_v, &s->grad})
        if (e == hipSuccess) e = hipMemcpy(*p, zero.data(), N_PARAMS * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        surrogate_free(s);
        return e;
    }
    *out = s;
    return hipSuccess;
}

static hipError_t pack_all(Surrogate *s, hipStream_t st)
{
    for (int l = 0; l < NL; ++l) {
        const int n = LKP[l] * LN[l];
        hipLaunchKernelGGL(k_pack_layer, dim3((n + 255) / 256), dim3(256), 0, st, s->master + layer_param_offset(l),
                           LK[l], LKP[l], LN[l], s->wt[l], s->wk[l], s->bias[l]);
    }
    return hipGetLastError();
}

hipError_t surrogate_set_state(Surrogate *s, const float *master, const float *m, const float *v, int64_t step)
{
    hipError_t e = hipMemcpy(s->master, master, N_PARAMS * 4, hipMemcpyHostToDevice);
    std::vector<float> zero;
    if (!m || !v) zero.assign(N_PARAMS, 0.f);
    if (e == hipSuccess) e = hipMemcpy(s->adam_m, m ? m : zero.data(), N_PARAMS * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->adam_v, v ? v : zero.data(), N_PARAMS * 4, hipMemcpyHostToDevice);
    s->step = step;
    if (e == hipSuccess) e = pack_all(s, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e;
}

hipError_t surrogate_get_state(const Surrogate *s, float *master, float *m, float *v, int64_t *step)
{
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && master) e = hipMemcpy(master, s->master, N_PARAMS * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && m) e = hipMemcpy(m, s->adam_m, N_PARAMS * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && v) e = hipMemcpy(v, s->adam_v, N_PARAMS * 4, hipMemcpyDeviceToHost);
    if (step) *step = s->step;
    return e;
}

hipError_t surrogate_set_norm(Surrogate *s, const float *mu, const float *sg)
{
    hipError_t e = hipMemcpy(s->mu, mu, NCOEF * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->sg, sg, NCOEF * 4, hipMemcpyHostToDevice);
    return e;
}

hipError_t surrogate_set_loss_weights(Surrogate *s, const float *w)
{
    std::vector<float> one(NCOEF, 1.f);
    return hipMemcpy(s->lw, w ? w : one.data(), NCOEF * 4, hipMemcpyHostToDevice);
}

template <bool TA, bool TB, int EPI>
static void gemm(const __bf16 *A, int lda, const __bf16 *B, int ldb, int K, int kchunk, int split, const float *bias,
                 const __bf16 *mask, int ldm, void *out, int ldo, int M, int N, hipStream_t st)
{
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), dim3(N / TN, M / TM, split), dim3(256), 0, st, A, lda, B, ldb, K, kchunk,
                       bias, mask, ldm, out, ldo, M, N);
}

static void forward_layers(Surrogate *s, const float *gbuf, const float *geo, int n_img, int H, int W, hipStream_t st)
{
    const int64_t rows = (int64_t)n_img * H * W;
    hipLaunchKernelGGL(k_im2col, dim3((unsigned)((rows * 9 + 255) / 256)), dim3(256), 0, st, gbuf, n_img, H, W,
                       s->x[0]);
    hipLaunchKernelGGL(k_geo_cols, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, gbuf, geo, n_img, H, W,
                       s->r_max, s->x[0]);
    for (int l = 0; l < NL; ++l) {
        if (l < NL - 1)
            gemm<false, false, EPI_BIAS_RELU>(s->x[l], LKP[l], s->wt[l], LKP[l], LKP[l], LKP[l], 1, s->bias[l],
                                              nullptr, 0, s->x[l + 1], LKP[l + 1], (int)rows, LN[l], st);
        else
            gemm<false, false, EPI_BIAS>(s->x[l], LKP[l], s->wt[l], LKP[l], LKP[l], LKP[l], 1, s->bias[l], nullptr, 0,
                                         s->y, NCOEF, (int)rows, LN[l], st);
    }
}

// Inference: one fused launch (rows a multiple of MLP_ROWS, checked by the caller).
hipError_t surrogate_forward(Surrogate *s, const float *gbuf, const float *geo, int n_img, int H, int W, float *coef,
                             hipStream_t st)
{
    const int64_t rows = (int64_t)n_img * H * W;
    MlpWeights w;
    for (int l = 0; l < NL; ++l) {
        w.wt[l] = s->wt[l];
        w.bias[l] = s->bias[l];
    }
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)(rows / MLP_ROWS)), dim3(256), 0, st, gbuf, geo, H, W, s->r_max,
                       w, coef);
    return hipGetLastError();
}

// Forward, loss and backward into s->grad; returns the loss on the device.
static hipError_t gradient(Surrogate *s, const float *gbuf, const float *geo, int n_img, int H, int W,
                           const float *target, float *dev_loss, hipStream_t st)
{
    const int64_t rows = (int64_t)n_img * H * W;
    forward_layers(s, gbuf, geo, n_img, H, W, st);
    const int64_t n = rows * NCOEF;
    const int nblk = (int)((n + 4095) / 4096);
    hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, st, s->y, target, s->lw, n, s->dz[0], s->dpart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, s->dpart, nblk, n, dev_loss);
    const int S = (int)((rows + SPLIT_ROWS - 1) / SPLIT_ROWS);
    int cur = 0;
    for (int l = NL - 1; l >= 0; --l) {
        const int K = LKP[l], N = LN[l];
        __bf16 *dzl = s->dz[cur];
        // weight gradient: X_l^T dZ_l, split over row chunks, then a fixed-order sum
        gemm<true, true, EPI_PARTIAL>(s->x[l], K, dzl, N, (int)rows, SPLIT_ROWS, S, nullptr, nullptr, 0, s->part, N, K,
                                      N, st);
        hipLaunchKernelGGL(k_reduce_partials, dim3((K * N + 255) / 256), dim3(256), 0, st, s->part, S, K, N, LK[l],
                           s->grad + layer_param_offset(l));
        // bias gradient: column sums of dZ_l
        hipLaunchKernelGGL(k_colsum, dim3(S, N / 64), dim3(256), 0, st, dzl, rows, N, s->part);
        hipLaunchKernelGGL(k_reduce_partials, dim3((N + 255) / 256), dim3(256), 0, st, s->part, S, 1, N, 1,
                           s->grad + layer_param_offset(l) + (int64_t)LK[l] * N);
        if (l > 0) {
            // dZ_{l-1} = (dZ_l W_l^T) masked by x_l > 0
            gemm<false, false, EPI_MASK>(dzl, N, s->wk[l], N, N, N, 1, nullptr, s->x[l], K, s->dz[cur ^ 1], K,
                                         (int)rows, K, st);
            cur ^= 1;
        }
    }
    return hipGetLastError();
}

hipError_t surrogate_gradient(Surrogate *s, const float *gbuf, const float *geo, int n_img, int H, int W,
                              const float *target, float *dev_grad, float *dev_loss, hipStream_t st)
{
    hipError_t e = gradient(s, gbuf, geo, n_img, H, W, target, dev_loss, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dev_grad, s->grad, N_PARAMS * 4, hipMemcpyDeviceToDevice, st);
    return e;
}

hipError_t surrogate_train_step(Surrogate *s, const float *gbuf, const float *geo, int n_img, int H, int W,
                                const float *target, float lr, float *dev_loss, hipStream_t st)
{
    hipError_t e = gradient(s, gbuf, geo, n_img, H, W, target, dev_loss, st);
    if (e != hipSuccess) return e;
    s->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - pow(0.9, (double)s->step)), c2 = (float)(1.0 - pow(0.999, (double)s->step));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((N_PARAMS + 255) / 256)), dim3(256), 0, st, s->master, s->adam_m,
                       s->adam_v, s->grad, N_PARAMS, lr, b1, b2, 1e-8f, c1, c2);
    return pack_all(s, st);
}

// Smooths i1 into s1 and, when given, im into sm.
static void smooth_channels(const Surrogate *s, const float *i1, const float *im, int64_t rows, hipStream_t st)
{
    const size_t lds = (size_t)2 * (s->n_bins + (s->n_bins >> 4) + 1) * sizeof(float);
    hipLaunchKernelGGL(k_smooth, dim3((unsigned)rows), dim3(64), lds, st, i1, im, s->n_bins, s->smooth, s->s1, s->sm);
}

hipError_t surrogate_target_coef(const Surrogate *s, const float *im, const float *gbuf, int64_t rows,
                                 int standardize, float *coef, hipStream_t st)
{
    smooth_channels(s, nullptr, im, rows, st);
    hipLaunchKernelGGL(k_level_coef, dim3((unsigned)((rows + 63) / 64)), dim3(256), 0, st, s->sm, gbuf, rows,
                       s->n_bins, s->r_min, s->r_max, s->basis, s->mu, s->sg, standardize, coef);
    return hipGetLastError();
}

hipError_t surrogate_coef_moments(Surrogate *s, const float *coef, int64_t rows, double *host_sum, double *host_sq,
                                  hipStream_t st)
{
    const int nb = (int)((rows + SPLIT_ROWS - 1) / SPLIT_ROWS);
    hipLaunchKernelGGL(k_coef_moments, dim3(nb), dim3(256), 0, st, coef, rows, s->dpart);
    std::vector<double> h((size_t)nb * 128);
    hipError_t e = hipMemcpyAsync(h.data(), s->dpart, h.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int j = 0; j < 64; ++j) {
        double a = 0, b = 0;
        for (int q = 0; q < nb; ++q) {
            a += h[(size_t)q * 128 + j];
            b += h[(size_t)q * 128 + 64 + j];
        }
        host_sum[j] = a;
        host_sq[j] = b;
    }
    return hipSuccess;
}

hipError_t surrogate_profile_errors(const Surrogate *s, const float *pred, const float *i1, const float *im,
                                    const float *gbuf, int64_t rows, float *err, float *profile, hipStream_t st)
{
    // the errors against the smoothed truth need both channels smoothed; the
    // profile itself uses the raw single-bounce channel
    if (im) smooth_channels(s, i1, im, rows, st);
    if (im)
        hipLaunchKernelGGL(k_mean_level, dim3((unsigned)((s->n_bins + 255) / 256)), dim3(256), 0, st, s->basis,
                           s->mu, s->n_bins, s->mlev);
    const size_t lds = (size_t)PR_ROWS * (s->n_bins + 1) * sizeof(float);
    const int per = (s->n_bins + 255) / 256;
#define SONAR_PROFILE(PP)                                                                                        \
    hipLaunchKernelGGL(k_profile_errors<PP>, dim3((unsigned)((rows + PR_ROWS - 1) / PR_ROWS)), dim3(256), lds, st, \
                       pred, i1, im, s->s1, s->sm, gbuf, rows, s->n_bins, s->r_min, s->r_max, s->mu, s->sg, s->mlev, \
                       err, profile)
    if (per <= 1) SONAR_PROFILE(1);
    else if (per <= 2) SONAR_PROFILE(2);
    else if (per <= 4) SONAR_PROFILE(4);
    else SONAR_PROFILE(8);
#undef SONAR_PROFILE
    return hipGetLastError();
}

int64_t surrogate_max_rows(const Surrogate *s) { return s->max_rows; }
int surrogate_bins(const Surrogate *s) { return s->n_bins; }

}  // namespace sonar
