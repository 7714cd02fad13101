// lm_peak.hip -- device micro-benchmarks used to calibrate the roofline of the
// shooting kernel: the issue rate of plain (unpacked) FP32 FMAs, of the
// ray-lens pair instruction mix (sub, fma, rcp, mul, fma, fma), and of single
// instruction kinds (VOP2 mul and fmac, VOP3 fma, rcp) and the kernel's
// shared-reciprocal pair pattern.
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

// Issue-rate probes: 8 independent chains per lane of one instruction kind, 4
// instructions per chain and iteration.  MODE 0: v_mul_f32 (VOP2); 1: v_fmac_f32
// (VOP2, accumulator form); 2: v_fma_f32 with a scalar operand (VOP3); 3:
// v_rcp_f32; 4: the shooting kernel's pair pattern, two columns sharing one
// reciprocal (add, add, mul, rcp, mul, mul, 4 fmac per two pairs).
// FP64 issue probe: 8 independent v_fma_f64 accumulator chains per lane, 4
// instructions per chain and iteration (the coefficient kernel's and the FP64
// near-sum mode's workhorse).
__global__ __launch_bounds__(256) void k_issue_f64(float* out, int iters)
{
    double a[kChains], b[kChains], x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        a[k] = 1.0 + 1e-3 * (double)threadIdx.x + (double)k;
        b[k] = 0.999 - 1e-4 * (double)k;
        x[k] = 1.0 + 0.01 * (double)k;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
#pragma unroll
            for (int u = 0; u < 4; ++u) x[k] = __builtin_fma(a[k], u & 1 ? b[k] : -b[k], x[k]);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    if (s == 1234.5) out[threadIdx.x] = (float)s;  // keeps the chains alive
}

template <int MODE>
__global__ __launch_bounds__(256) void k_issue(float* out, int iters, float s0, float s1)
{
    float a[kChains], b[kChains], x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        a[k] = 1.0f + 1e-3f * (float)threadIdx.x + (float)k;
        b[k] = 0.999f - 1e-4f * (float)k;
        x[k] = 1.0f + 0.01f * (float)k;
    }
    float dy2 = 0.3f + 1e-4f * (float)threadIdx.x, mdy = 0.1f;
    for (int i = 0; i < iters; ++i) {
        if (MODE == 4) {
#pragma unroll
            for (int k = 0; k < kChains; k += 2) {
                const float r2a = a[k] + dy2, r2b = a[k + 1] + dy2;
                const float r = __builtin_amdgcn_rcpf(r2a * r2b);
                const float wa = r * r2b, wb = r * r2a;
                x[k] = __builtin_fmaf(b[k], wa, x[k]);
                x[k + 1] = __builtin_fmaf(mdy, wa, x[k + 1]);
                b[k + 1] = __builtin_fmaf(b[k], wb, b[k + 1]);
                a[k] = __builtin_fmaf(mdy, wb, a[k]);
            }
            dy2 = dy2 + s1;
        } else {
#pragma unroll
            for (int k = 0; k < kChains; ++k) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (MODE == 0) x[k] = x[k] * (u & 1 ? a[k] : b[k]);
                    if (MODE == 1) x[k] = __builtin_fmaf(a[k], b[k], x[k]);
                    if (MODE == 2) x[k] = __builtin_fmaf(x[k], u & 1 ? s1 : s0, a[k]);
                    if (MODE == 3) x[k] = __builtin_amdgcn_rcpf(x[k]);
                }
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k] + a[k] + b[k];
    if (s == 1234.5f) out[threadIdx.x] = s;  // keeps the chains alive
}

template <int MODE>
float time_issue(dim3 grid, float* out, int iters, hipEvent_t e0, hipEvent_t e1)
{
    // MODE 5: the FP64 probe
    for (int rep = 0; rep < 2; ++rep) {
        if (rep == 1) (void)hipEventRecord(e0, nullptr);
        if constexpr (MODE == 5)
            hipLaunchKernelGGL(k_issue_f64, grid, dim3(256), 0, nullptr, out, iters);
        else
            hipLaunchKernelGGL(k_issue<MODE>, grid, dim3(256), 0, nullptr, out, iters, 0.999f,
                               1e-3f);
    }
    (void)hipEventRecord(e1, nullptr);
    float ms = -1.f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return -1.f;
    return ms;
}

}  // namespace

extern "C" lm_status lm_measure_issue_rates(double* rates, int32_t n)
{
    if (!rates || n < 0) return LM_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return LM_EDEVICE;
    float* out = nullptr;
    if (hipMalloc(&out, 256 * sizeof(float)) != hipSuccess) return LM_ENOMEM;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int iters = 1 << 11;
    const dim3 grid(cus * 16);
    const double lanes = (double)grid.x * 256;
    float ms[6];
    ms[0] = time_issue<0>(grid, out, iters, e0, e1);
    ms[1] = time_issue<1>(grid, out, iters, e0, e1);
    ms[2] = time_issue<2>(grid, out, iters, e0, e1);
    ms[3] = time_issue<3>(grid, out, iters, e0, e1);
    ms[4] = time_issue<4>(grid, out, iters, e0, e1);
    ms[5] = time_issue<5>(grid, out, iters, e0, e1);
    lm_status st = LM_OK;
    for (int k = 0; k < 6; ++k) {
        if (ms[k] <= 0.f) {
            st = LM_EDEVICE;
            break;
        }
        // modes 0-3 and 5: lane instructions per second; mode 4: near pairs per second
        const double units = k != 4 ? lanes * iters * kChains * 4 : lanes * iters * kChains;
        if (k < n) rates[k] = units / (ms[k] * 1e-3);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return st;
}

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
