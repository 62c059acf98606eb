// Pulse compression of the echo volume (Sec. II-B: time-series data next to
// the intensity volumes, for matched filtering). A beam's complex range
// column x[n] is the impulse response at the bins' two-way delay spacing; the
// received baseband series is its convolution with the transmitted pulse,
// s[n] = sum_k p[k] x[n-k], and the matched-filter output correlates the
// series with the pulse, y[n] = sum_k conj(p[k]) s[n+k], both over the record
// [0, N) with zeros outside.
//
// k_pulse: one block per beam. The column goes to LDS behind 64 zeros, the
// series is formed there (and written out if requested), followed by 68
// zeros, then the matched output is formed from it. Each thread computes four
// consecutive outputs with a sliding window of four samples in registers:
// one LDS read and four complex multiply-adds per pulse tap. HBM traffic per
// beam: the column once, each requested output once. The taps travel in the
// kernel arguments (uniform scalar loads), so a launch allocates nothing.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace sonar {

namespace {

constexpr int XPAD = 64;                // zeros before the column: x[n - k] for k < 64
constexpr int SPAD = 68;                // zeros after the series: s[n + k] for a window of 4 and k < 64

__device__ __forceinline__ void cmac(float2 &acc, const float2 p, const float2 v)
{
    acc.x = fmaf(p.x, v.x, acc.x);
    acc.x = fmaf(-p.y, v.y, acc.x);
    acc.y = fmaf(p.x, v.y, acc.y);
    acc.y = fmaf(p.y, v.x, acc.y);
}

__device__ __forceinline__ void cmac_conj(float2 &acc, const float2 p, const float2 v)
{
    acc.x = fmaf(p.x, v.x, acc.x);
    acc.x = fmaf(p.y, v.y, acc.x);
    acc.y = fmaf(p.x, v.y, acc.y);
    acc.y = fmaf(-p.y, v.x, acc.y);
}

// A staged row from LDS to its output: consecutive lanes take consecutive
// pairs of samples (one 16-byte store each when the row starts 16-byte
// aligned), with non-temporal stores, since nothing here reads them again.
__device__ __forceinline__ void stream_out(const float2 *__restrict__ src, float2 *__restrict__ dst, int N, int t,
                                           int T)
{
    typedef float f4v __attribute__((ext_vector_type(4)));
    typedef float f2v __attribute__((ext_vector_type(2)));
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        for (int i = t; i < N / 2; i += T)
            __builtin_nontemporal_store(f4v{src[2 * i].x, src[2 * i].y, src[2 * i + 1].x, src[2 * i + 1].y},
                                        reinterpret_cast<f4v *>(dst) + i);
        if ((N & 1) && t == 0) __builtin_nontemporal_store(f2v{src[N - 1].x, src[N - 1].y}, reinterpret_cast<f2v *>(dst) + N - 1);
    } else {
        for (int i = t; i < N; i += T)
            __builtin_nontemporal_store(f2v{src[i].x, src[i].y}, reinterpret_cast<f2v *>(dst) + i);
    }
}

__global__ __launch_bounds__(256) void k_pulse(PulseArgs a)
{
    extern __shared__ float2 lds_c[];
    const int N = a.n_bins, L = a.L, T = blockDim.x, t = threadIdx.x;
    float2 *xl = lds_c;                 // x[i] at xl[XPAD + i]
    float2 *sl = lds_c + XPAD + N;      // s[i] at sl[i], zeros in [N, N + SPAD)
    const size_t base = (size_t)blockIdx.x * (size_t)N;
    const float2 zero = make_float2(0.f, 0.f);
    for (int i = t; i < N; i += T) xl[XPAD + i] = a.x[base + i];
    for (int i = t; i < XPAD; i += T) xl[i] = zero;
    for (int i = t; i < SPAD; i += T) sl[N + i] = zero;
    __syncthreads();

    for (int n0 = 4 * t; n0 < N; n0 += 4 * T) {
        // window w_j = x[n0 + j - k], starting at k = 0
        // (samples past the record stay zero: their outputs are not stored)
        float2 w0 = xl[XPAD + n0];
        float2 w1 = n0 + 1 < N ? xl[XPAD + n0 + 1] : zero;
        float2 w2 = n0 + 2 < N ? xl[XPAD + n0 + 2] : zero;
        float2 w3 = n0 + 3 < N ? xl[XPAD + n0 + 3] : zero;
        float2 c0 = zero, c1 = zero, c2 = zero, c3 = zero;
        for (int k = 0; k < L; ++k) {
            const float2 p = a.p[k];
            cmac(c0, p, w0);
            cmac(c1, p, w1);
            cmac(c2, p, w2);
            cmac(c3, p, w3);
            w3 = w2;
            w2 = w1;
            w1 = w0;
            w0 = xl[XPAD + n0 - k - 1];
        }
        const float2 c[4] = {c0, c1, c2, c3};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (n0 + j < N) sl[n0 + j] = c[j];
    }
    __syncthreads();
    if (a.s) stream_out(sl, a.s + base, N, t, T);
    if (!a.y) return;

    for (int n0 = 4 * t; n0 < N; n0 += 4 * T) {
        // window w_j = s[n0 + j + k], starting at k = 0
        float2 w0 = sl[n0], w1 = sl[n0 + 1], w2 = sl[n0 + 2], w3 = sl[n0 + 3];
        float2 c0 = zero, c1 = zero, c2 = zero, c3 = zero;
        for (int k = 0; k < L; ++k) {
            const float2 p = a.p[k];
            cmac_conj(c0, p, w0);
            cmac_conj(c1, p, w1);
            cmac_conj(c2, p, w2);
            cmac_conj(c3, p, w3);
            w0 = w1;
            w1 = w2;
            w2 = w3;
            w3 = sl[n0 + 4 + k];
        }
        const float2 c[4] = {c0, c1, c2, c3};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (n0 + j < N) xl[n0 + j] = c[j];          // the input is no longer needed
    }
    __syncthreads();
    stream_out(xl, a.y + base, N, t, T);
}

}  // namespace

int pulse_threads(int n_bins)
{
    int t = ((n_bins + 3) / 4 + 63) / 64 * 64;
    return t < 64 ? 64 : (t > 256 ? 256 : t);
}

size_t pulse_lds_bytes(int n_bins) { return sizeof(float2) * (size_t)(XPAD + 2 * n_bins + SPAD); }

hipError_t launch_pulse(const PulseArgs &a, hipStream_t s)
{
    if (a.n_beams == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pulse, dim3((unsigned)a.n_beams), dim3(pulse_threads(a.n_bins)), pulse_lds_bytes(a.n_bins),
                       s, a);
    return hipGetLastError();
}

}  // namespace sonar
