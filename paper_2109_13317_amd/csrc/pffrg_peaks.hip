// pffrg_peaks.hip -- on-device measurement of the peaks the kernels are
// judged against: FP64 and FP32 vector FMA throughput (no packed FP32, as in
// every kernel of the library), device-memory copy bandwidth, and the rates
// at which 16-byte-per-lane loads (one interpolation corner of a pair) come
// from L1 and from LDS.  A diagnostic; nothing in the flow depends on it.
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

// 16 bytes per lane per load, kLoadIters loads per lane.  L1: 128-bit raw
// buffer loads from a 16 KB buffer (L1-resident after the first pass), each
// wave instruction one contiguous 1 KB row, or (two_rows) two 512-byte rows,
// the shape of two pair vectors per instruction.  LDS: 128-bit reads of a
// 16 KB LDS copy, one contiguous 1 KB row per wave instruction.  Row
// positions come from a hash of the wave and the iteration (wave-uniform,
// never periodic, so no load can be hoisted out of the loop) and are masked
// into the buffer; the loaded values are summed and stored so the loads are
// kept.
constexpr int kLoadIters = 4096;
constexpr int kLoadBufBytes = 16384;

__device__ __forceinline__ unsigned row_hash(unsigned wave, unsigned i) {
    unsigned h = wave * 0x9E3779B1u + i * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 13;
    return h;
}

__global__ void __launch_bounds__(kPeakThreads) k_l1_rate(const double2* __restrict__ buf, int two_rows,
                                                          double* __restrict__ out) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)buf, (short)0, kLoadBufBytes, 0x00020000);
    const int lane = threadIdx.x & 63;
    const unsigned wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const unsigned half = two_rows ? (unsigned)(lane >> 5) : 0u;
    const unsigned col = two_rows ? (unsigned)(lane & 31) * 16u : (unsigned)lane * 16u;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < kLoadIters; i += 4)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned h = row_hash(wave, (unsigned)(i + j));
            const unsigned rowb = two_rows ? ((half ? (h >> 16) : h) & 0x3FFu) * 16u : (h & 0x3FFu) * 16u;
            const unsigned o = (rowb + col) & (unsigned)(kLoadBufBytes - 16);
            const double2 g = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)o, 0, 0));
            a[j] += g.x + g.y;
        }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a[0] + a[1] + a[2] + a[3];
}

__global__ void __launch_bounds__(kPeakThreads) k_lds_rate(const double2* __restrict__ buf, double* __restrict__ out) {
    constexpr int n = kLoadBufBytes / 16;
    __shared__ double2 s[n];
    for (int i = threadIdx.x; i < n; i += kPeakThreads) s[i] = buf[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const unsigned wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < kLoadIters; i += 4)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned h = row_hash(wave, (unsigned)(i + j));
            const double2 g = s[((h & 0x3FFu) + (unsigned)lane) & (unsigned)(n - 1)];
            a[j] += g.x + g.y;
        }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a[0] + a[1] + a[2] + a[3];
}

// TB/s of 16-byte lane loads by kind: 0 L1 one row, 1 L1 two rows, 2 LDS.
pffrg_status load_rate(hipStream_t s, const double2* buf, double* out, hipEvent_t e0, hipEvent_t e1, int kind,
                       double* tbs) {
    float best = 0.0f;
    for (int rep = 0; rep < 3; ++rep) {
        HIP_TRY(hipEventRecord(e0, s));
        if (kind < 2) hipLaunchKernelGGL(k_l1_rate, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, buf, kind, out);
        else hipLaunchKernelGGL(k_lds_rate, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, buf, out);
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0 && (best == 0.0f || ms < best)) best = ms;      // the first launch warms the caches
    }
    TRY(launch_check(kind < 2 ? "k_l1_rate" : "k_lds_rate"));
    *tbs = 16.0 * kLoadIters * (double)kPeakBlocks * kPeakThreads / (best * 1e-3) / 1e12;
    return PFFRG_OK;
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
    // 16-byte lane loads: the copy's source (zeros) serves as the 16 KB buffer
    const double2* lb = reinterpret_cast<const double2*>(src);
    TRY(load_rate(stream, lb, o64, e0, e1, 0, &out->l1_load_tbs));
    TRY(load_rate(stream, lb, o64, e0, e1, 1, &out->l1_load_2row_tbs));
    TRY(load_rate(stream, lb, o64, e0, e1, 2, &out->lds_read_tbs));
    HIP_TRY(hipStreamSynchronize(stream));
    return PFFRG_OK;
}
