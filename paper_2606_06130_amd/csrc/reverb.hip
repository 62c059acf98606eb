// Water-column volume reverberation and receiver noise (Sec. II-B: volumetric
// backscatter from the water column; speckle). Every range cell of a
// cell-centred beam layout receives a circular complex Gaussian sample whose
// mean power is s_v V / r^4 10^(-alpha 2 r / 10) + N0, V = r^2 cos(el)
// dth_h dth_v dr the cell's volume at its centre range r and elevation el.
// The sample is sqrt(P / 2) sqrt(-2 ln u1) e^(2 pi i u2) (Box-Muller) with
// u1 = (top 24 bits + 1) / 2^24 and u2 = the next 24 bits / 2^24 of
// SplitMix64(seed, c + 1), c = (ping << 43) ^ (beam << 12) ^ bin, so every
// cell's sample is fixed by its indices (no state, any launch order).
//
// k_reverb: grid x = beams, grid y = chunks of 256 bins; one cell per thread,
// read-modify-write of the volume (HBM-bound: 16 bytes per cell).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace sonar {

namespace {

__global__ __launch_bounds__(256) void k_reverb(ReverbArgs a)
{
    const int64_t b = blockIdx.x;
    const int n = blockIdx.y * 256 + threadIdx.x;
    // the beam's factor s_v cos(el) dth_h dth_v dr is the same for the whole
    // block: one lane evaluates it (the kernel is as much ALU- as HBM-bound)
    __shared__ float beam_k;
    if (threadIdx.x == 0) {
        const int v = (int)(b / a.beams_h);
        const float el = -0.5f * a.vfov + ((float)v + 0.5f) * a.dth_v;
        beam_k = a.sv * cosf(el) * a.cell_solid * a.dr;
    }
    __syncthreads();
    if (n >= a.n_bins) return;
    const float r = a.r_min + ((float)n + 0.5f) * a.dr;
    const float P = beam_k / (r * r) * exp10f(-0.2f * a.alpha_db * r) + a.noise;
    const uint64_t c = ((uint64_t)a.ping << 43) ^ ((uint64_t)b << 12) ^ (uint64_t)n;
    const uint64_t z = splitmix64_nth(a.seed, c + 1);
    const float u1 = (float)((z >> 40) + 1) * (1.f / 16777216.f);
    const float u2 = (float)((z >> 16) & 0xFFFFFFull) * (1.f / 16777216.f);
    float sn, cs;
    sincospif(2.f * u2, &sn, &cs);
    const float amp = sqrtf(-P * logf(u1));      // sqrt(P / 2) sqrt(-2 ln u1)
    typedef float f2v __attribute__((ext_vector_type(2)));
    f2v *cell = reinterpret_cast<f2v *>(a.volume) + b * a.n_bins + n;
    const f2v e = *cell;
    __builtin_nontemporal_store(f2v{fmaf(amp, cs, e.x), fmaf(amp, sn, e.y)}, cell);     // streamed back out
}

}  // namespace

hipError_t launch_reverb(const ReverbArgs &a, hipStream_t s)
{
    if (a.n_beams == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reverb, dim3((unsigned)a.n_beams, (unsigned)((a.n_bins + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sonar
