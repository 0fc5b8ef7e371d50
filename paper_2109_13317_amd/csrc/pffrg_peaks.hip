// pffrg_peaks.hip -- on-device measurement of the peaks the kernels are
// judged against: FP64 and FP32 vector FMA throughput (no packed FP32, as in
// every kernel of the library) and device-memory copy bandwidth.  A
// diagnostic; nothing in the flow depends on it.
#include <hip/hip_runtime.h>

#include "pffrg.h"
#include "host_common.h"

using namespace pffrg_host;

namespace {

constexpr int kChains = 8;        // independent FMA chains per lane (hide the FMA latency)
constexpr int kPeakBlocks = 256 * 8;
constexpr int kPeakThreads = 256;

// Each lane runs kChains dependent FMA chains for n rounds; the result is
// stored so the work is kept.
template <class T>
__global__ void __launch_bounds__(kPeakThreads) k_fma_rate(int n, T b, T c, T* __restrict__ out) {
    T a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = (T)(threadIdx.x + i);
    for (int r = 0; r < n; ++r)
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = fma(a[i], b, c);
    T s = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_copy(long n, const double4* __restrict__ src, double4* __restrict__ dst) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

template <class T>
pffrg_status fma_rate(hipStream_t s, T* out, hipEvent_t e0, hipEvent_t e1, double* tflops) {
    const int n = 4096;
    // b slightly below 1 and c = 0 keep the chains finite and normal
    hipLaunchKernelGGL(k_fma_rate<T>, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, 64, (T)0.999, (T)0, out);
    HIP_TRY(hipEventRecord(e0, s));
    hipLaunchKernelGGL(k_fma_rate<T>, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, n, (T)0.999, (T)0, out);
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    *tflops = 2.0 * kChains * (double)n * kPeakBlocks * kPeakThreads / (ms * 1e-3) / 1e12;
    return launch_check("k_fma_rate");
}

// Buffers and events of one measurement, released on every return path.
struct Scratch {
    DevAllocs mem;
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Scratch() {
        for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
        mem.release();
    }
};

}  // namespace

extern "C" pffrg_status pffrg_measure_peaks(void* stream_ptr, pffrg_peaks* out) {
    if (!out) return fail(PFFRG_EINVAL, "null output");
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    Scratch sc;
    DevAllocs& mem = sc.mem;
    double* o64 = nullptr;
    TRY(mem.alloc(&o64, (size_t)kPeakBlocks * kPeakThreads));
    float* o32 = nullptr;
    TRY(mem.alloc(&o32, (size_t)kPeakBlocks * kPeakThreads));
    HIP_TRY(hipEventCreate(&sc.e[0]));
    HIP_TRY(hipEventCreate(&sc.e[1]));
    hipEvent_t e0 = sc.e[0], e1 = sc.e[1];
    TRY(fma_rate<double>(stream, o64, e0, e1, &out->fp64_fma_tflops));
    TRY(fma_rate<float>(stream, o32, e0, e1, &out->fp32_fma_tflops));
    // copy bandwidth: 512 MiB read and 512 MiB written per pass
    const long n4 = (512L << 20) / (long)sizeof(double4);
    double4 *src = nullptr, *dst = nullptr;
    TRY(mem.alloc(&src, (size_t)n4));
    TRY(mem.alloc(&dst, (size_t)n4));
    HIP_TRY(hipMemsetAsync(src, 0, sizeof(double4) * n4, stream));
    const int grid = 256 * 16;
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, stream, n4, (const double4*)src, dst);
    HIP_TRY(hipEventRecord(e0, stream));
    for (int r = 0; r < 5; ++r)
        hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, stream, n4, (const double4*)src, dst);
    HIP_TRY(hipEventRecord(e1, stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    TRY(launch_check("k_copy"));
    HIP_TRY(hipStreamSynchronize(stream));
    out->hbm_copy_gbs = 5.0 * 2.0 * sizeof(double4) * (double)n4 / (ms * 1e-3) / 1e9;
    return PFFRG_OK;
}
