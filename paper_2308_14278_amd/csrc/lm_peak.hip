// lm_peak.hip -- device micro-benchmarks used to calibrate the roofline of the
// shooting kernel: the issue rate of plain (unpacked) FP32 FMAs, and of the
// ray-lens pair instruction mix (sub, fma, rcp, mul, fma, fma).
#include <hip/hip_runtime.h>

#include "../../include/lensmap.h"

namespace {

constexpr int kChains = 8;

__global__ __launch_bounds__(256) void k_fma_peak(float* out, int iters, float b, float c)
{
    float a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = (float)(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = __builtin_fmaf(a[k], b, c);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    if (s == 1234.5f) out[threadIdx.x] = s;  // keeps the chains alive
}

// The per-pair mix of the near-lens loop: dx = px - lx; r2 = fma(dx, dx, dy2);
// w = m * rcp(r2); ax = fma(dx, w, ax); ay = fma(dy, w, ay).
__global__ __launch_bounds__(256) void k_pair_peak(float* out, int iters, float lx, float m)
{
    float px[kChains], ax[kChains], ay[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        px[k] = 0.01f * (float)(threadIdx.x + 3 * k) + 1.0f;
        ax[k] = 0.f;
        ay[k] = 0.f;
    }
    const float dy = 0.37f + 1e-3f * (float)threadIdx.x, dy2 = dy * dy;
    for (int i = 0; i < iters; ++i) {
        const float l = lx + 1e-6f * (float)i;
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            const float dx = px[k] - l;
            const float r2 = __builtin_fmaf(dx, dx, dy2);
            const float w = m * __builtin_amdgcn_rcpf(r2);
            ax[k] = __builtin_fmaf(dx, w, ax[k]);
            ay[k] = __builtin_fmaf(dy, w, ay[k]);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += ax[k] + ay[k];
    if (s == 1234.5f) out[threadIdx.x] = s;
}

}  // namespace

extern "C" lm_status lm_measure_valu_peak(double* fma_tflops, double* pair_gpairs)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return LM_EDEVICE;
    float* out = nullptr;
    if (hipMalloc(&out, 256 * sizeof(float)) != hipSuccess) return LM_ENOMEM;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int iters = 1 << 14;
    const dim3 grid(cus * 8), block(256);
    float ms = 0.f;
    lm_status st = LM_OK;
    // warm-up, then timed runs
    hipLaunchKernelGGL(k_fma_peak, grid, block, 0, nullptr, out, iters, 0.999f, 1e-3f);
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(k_fma_peak, grid, block, 0, nullptr, out, iters, 0.999f, 1e-3f);
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        st = LM_EDEVICE;
    if (fma_tflops && st == LM_OK)
        *fma_tflops = 2.0 * kChains * (double)iters * grid.x * block.x / (ms * 1e-3) / 1e12;
    hipLaunchKernelGGL(k_pair_peak, grid, block, 0, nullptr, out, iters / 4, 0.5f, 0.3f);
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(k_pair_peak, grid, block, 0, nullptr, out, iters / 4, 0.5f, 0.3f);
    (void)hipEventRecord(e1, nullptr);
    if (st == LM_OK &&
        (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = LM_EDEVICE;
    if (pair_gpairs && st == LM_OK)
        *pair_gpairs = (double)kChains * (iters / 4) * grid.x * block.x / (ms * 1e-3) / 1e9;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return st;
}
