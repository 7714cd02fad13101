// lm_analysis.hip -- light-curve peak identification on a count map (Sec. 4.2).
//
// A light curve is row i of the row-major map counts[i][j] (fixed source index
// along the caustic, j across it).  Candidate peak: N_ij > max(N_i,j-1, N_i,j+1)
// and h_ij > k sigma_ij with h_ij = N_ij - <N>, <N> the mean of the three
// counts and sigma_ij = sqrt(<N>); with S the sum of the three counts this is
// (3 N_ij - S)^2 > 3 k^2 S, decided exactly in integers.  True peak: a
// candidate with a candidate among (i-1, j-1..j+1) and among (i+1, j-1..j+1).
//
// k_peak_bins gathers the statistics of Sec. 4.2 (Figs. 4 and 5): the true
// peaks of the listed light curves per bin of distance to the caustic (bin of
// pixel j given by the host) and the sum of their counts, both exact integers.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>

#include "lm_internal.h"

namespace {

// Scratch memory of the allocation-free peak statistics: the listed rows, the
// bin of every pixel column and the two histograms, at fixed offsets.  Each
// device holds its own copy; host code reaches it only through the address
// hipGetSymbolAddress returns on that device.
static __device__ __align__(256) unsigned char scratch[LM_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[LM_MAX_DEVICES] = {};

__device__ __forceinline__ bool candidate(const unsigned long long* __restrict__ c, int64_t nx,
                                          int64_t i, int64_t j, unsigned k2x3)
{
    if (j <= 0 || j >= nx - 1) return false;
    const unsigned long long* row = c + i * nx;
    const unsigned long long a = row[j - 1], n = row[j], b = row[j + 1];
    if (!(n > a && n > b)) return false;
    const unsigned __int128 s = (unsigned __int128)a + n + b;
    const unsigned __int128 n3 = (unsigned __int128)n * 3u;
    if (n3 <= s) return false;
    const unsigned __int128 t = n3 - s;
    // 3 k^2 S < 2^90 for k <= 1000, so any t >= 2^64 passes
    if ((unsigned long long)(t >> 64) != 0ull) return true;
    const unsigned long long tl = (unsigned long long)t;
    return (unsigned __int128)tl * tl > (unsigned __int128)k2x3 * s;
}

__global__ __launch_bounds__(256) void k_peaks(const unsigned long long* __restrict__ counts,
                                               int64_t nx, int64_t ny,
                                               const int32_t* __restrict__ tracks, int64_t nt,
                                               unsigned k2x3, uint8_t* __restrict__ flags)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= nt * nx) return;
    const int64_t t = idx / nx, j = idx - t * nx;
    const int64_t i = tracks[t];
    uint8_t f = 0;
    if (candidate(counts, nx, i, j, k2x3)) {
        f = 1;
        if (i > 0 && i < ny - 1) {
            const bool left = candidate(counts, nx, i - 1, j - 1, k2x3) ||
                              candidate(counts, nx, i - 1, j, k2x3) ||
                              candidate(counts, nx, i - 1, j + 1, k2x3);
            const bool right = candidate(counts, nx, i + 1, j - 1, k2x3) ||
                               candidate(counts, nx, i + 1, j, k2x3) ||
                               candidate(counts, nx, i + 1, j + 1, k2x3);
            if (left && right) f |= 2;
        }
    }
    flags[idx] = f;
}

__device__ __forceinline__ bool true_peak(const unsigned long long* __restrict__ c, int64_t nx,
                                          int64_t ny, int64_t i, int64_t j, unsigned k2x3)
{
    if (!(i > 0 && i < ny - 1) || !candidate(c, nx, i, j, k2x3)) return false;
    const bool left = candidate(c, nx, i - 1, j - 1, k2x3) || candidate(c, nx, i - 1, j, k2x3) ||
                      candidate(c, nx, i - 1, j + 1, k2x3);
    return left && (candidate(c, nx, i + 1, j - 1, k2x3) || candidate(c, nx, i + 1, j, k2x3) ||
                    candidate(c, nx, i + 1, j + 1, k2x3));
}

// Distance bin of every pixel column: the bin holding the column centre
// x0 + (p + 1/2) dx, with the multiply and the add rounded separately as the
// host computes the same centres.
__global__ __launch_bounds__(256) void k_column_bins(double x0, double dx, int64_t nx,
                                                     const double* __restrict__ edges, int nb,
                                                     int32_t* __restrict__ bin_of)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= nx) return;
    const double c = __dadd_rn(x0, __dmul_rn((double)p + 0.5, dx));
    int b = -1;
    if (c >= edges[0] && c < edges[nb]) {
        int lo = 0, hi = nb - 1;  // the largest b with edges[b] <= c
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (edges[mid] <= c)
                lo = mid;
            else
                hi = mid - 1;
        }
        b = lo;
    }
    bin_of[p] = b;
}

// One thread per (light curve t, pixel j); true peaks are rare, so their bins
// are added to with global atomics.
__global__ __launch_bounds__(256) void k_peak_bins(const unsigned long long* __restrict__ counts,
                                                   int64_t nx, int64_t ny,
                                                   const int32_t* __restrict__ tracks, int64_t nt,
                                                   unsigned k2x3, const int32_t* __restrict__ bin_of,
                                                   unsigned long long* __restrict__ peaks,
                                                   unsigned long long* __restrict__ heights)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= nt * nx) return;
    const int64_t t = idx / nx, j = idx - t * nx;
    const int b = bin_of[j];
    if (b < 0) return;
    const int64_t i = tracks[t];
    if (!true_peak(counts, nx, ny, i, j, k2x3)) return;
    atomicAdd(&peaks[b], 1ull);
    atomicAdd(&heights[b], counts[i * nx + j]);
}

}  // namespace

int lm_launch_column_bins(double x0, double dx, int64_t nx, const double* edges, int nb,
                          int32_t* bin_of, void* stream)
{
    if (nx <= 0) return 0;
    hipLaunchKernelGGL(k_column_bins, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, x0, dx, nx, edges, nb, bin_of);
    return (int)hipGetLastError();
}

int lm_launch_peak_bins(const unsigned long long* counts, int64_t nx, int64_t ny,
                        const int32_t* tracks, int64_t nt, int k, const int32_t* bin_of,
                        unsigned long long* peaks, unsigned long long* heights, void* stream)
{
    const int64_t n = nt * nx;
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_peak_bins, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, counts, nx, ny, tracks, nt, (unsigned)(3 * k * k),
                       bin_of, peaks, heights);
    return (int)hipGetLastError();
}

int lm_launch_peaks(const unsigned long long* counts, int64_t nx, int64_t ny,
                    const int32_t* tracks, int64_t nt, int k, uint8_t* flags, void* stream)
{
    const int64_t n = nt * nx;
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_peaks, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, counts, nx, ny, tracks, nt, (unsigned)(3 * k * k),
                       flags);
    return (int)hipGetLastError();
}

int lm_scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= LM_MAX_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}
