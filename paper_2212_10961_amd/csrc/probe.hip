// Issue-rate probes for the benchmark: how many hardware cosines (v_cos_f32, argument in
// revolutions) the device completes per second in a register loop, alone and in the direct
// sum's per-term mix (one cosine, one add, one fused multiply-add).  The measured rates are
// reported beside the nominal half-rate figure derived from the unit counts and clock.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;  // independent dependency chains per lane

__global__ __launch_bounds__(256) void k_cos_only(float* out, int iters, float seed)
{
    float a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = seed + 1e-3f * threadIdx.x + 0.1f * c;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = __builtin_amdgcn_cosf(a[c]);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += a[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// One term of the direct sum: acc += w * cos(x + q) (x, q fractions, w a weight).
__global__ __launch_bounds__(256) void k_cos_mix(float* out, int iters, float seed)
{
    float acc[kChains], x[kChains];
    const float q = 0.37f + 1e-4f * threadIdx.x, w = 0.999f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        acc[c] = 0.f;
        x[c] = seed + 0.05f * c;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = fmaf(w, __builtin_amdgcn_cosf(x[c] + acc[c] * q), acc[c]);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

// Cosines per second of each probe (best of `reps` timed launches of `blocks` x 256 lanes,
// `iters` iterations of kChains cosines each).  `out` is device scratch of blocks * 256 floats.
// Returns 0, or a negative HIP error code.
extern "C" int grf_probe_cos_rates(float* out, int blocks, int iters, int reps, double* cos_only, double* cos_mix)
{
    if (!out || blocks < 1 || iters < 1 || reps < 1 || !cos_only || !cos_mix) return -1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -3;
    const double work = double(blocks) * 256.0 * double(iters) * kChains;
    double best[2] = {0.0, 0.0};
    int rc = 0;
    for (int k = 0; k < 2 && rc == 0; ++k) {
        for (int r = 0; r <= reps; ++r) {  // the first launch warms up
            hipEventRecord(e0, nullptr);
            if (k == 0) hipLaunchKernelGGL(k_cos_only, dim3(blocks), dim3(256), 0, nullptr, out, iters, 0.1f * r);
            else hipLaunchKernelGGL(k_cos_mix, dim3(blocks), dim3(256), 0, nullptr, out, iters, 0.1f * r);
            hipEventRecord(e1, nullptr);
            if (hipEventSynchronize(e1) != hipSuccess) {
                rc = -3;
                break;
            }
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            if (r > 0 && ms > 0.f && work / (ms * 1e-3) > best[k]) best[k] = work / (ms * 1e-3);
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *cos_only = best[0];
    *cos_mix = best[1];
    return rc;
}
