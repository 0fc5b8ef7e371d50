// pffrg_noalloc.hip -- the correlations chi_ij without a context and without
// device allocation (pffrg_chi_noalloc), for callers that cannot allocate.
//
// The chi kernels (kernels_obs.h) need a scratch area beside their inputs and
// outputs: the node list, trapezoid weights and squared propagators of the
// correlation integrals, the node count, and the per-slice partial double
// integrals of every pair.  pffrg_chi keeps it in its context; here it is the
// file-scope device array `scratch`, sized for the largest mesh and pair count
// the kernels take.  Each device holds its own copy of the array (for as long
// as the process runs); its device address is looked up once per device with
// hipGetSymbolAddress, and only that address is handed to kernels.  Every
// call on one device uses the same array, so calls that overlap on one device
// (two streams, or two host threads) race; a call writes every scratch entry
// it reads, so nothing has to be cleared between calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "pffrg.h"
#include "host_common.h"
#include "kernels_obs.h"

using namespace pffrg;
using namespace pffrg_host;

namespace {

// Layout of the scratch area in doubles: node frequencies cw, trapezoid
// weights cq and squared propagators cg2 (kNodes each), the node count (an
// int in one double slot), then the partial integrals [pairs][slices][2].
constexpr int kNodes = 2 * PFFRG_NOALLOC_MAX_FREQ + 4;
constexpr long kOffCw = 0, kOffCq = kNodes, kOffCg2 = 2L * kNodes, kOffCn = 3L * kNodes;
constexpr long kOffPart = kOffCn + 2;
constexpr long kScratchDoubles = kOffPart + (long)PFFRG_NOALLOC_MAX_PAIRS * kChiSlices * 2;
static_assert(PFFRG_NOALLOC_MAX_FREQ <= kMaxMesh, "k_chi_nodes stages at most kMaxMesh frequencies");
static_assert(kScratchDoubles * sizeof(double) == PFFRG_NOALLOC_SCRATCH_BYTES, "header states the scratch size");

}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current.  (The array's name in host code is a
// stand-in for registration, not a device address.)
pffrg_status scratch_address(double** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PFFRG_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PFFRG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return PFFRG_OK;
}

}  // namespace

extern "C" {

pffrg_status pffrg_chi_noalloc(int n_freq, const double* d_omega, int n_pairs, const int* d_swap, double lambda,
                               const double* d_state, double* d_chi, void* stream) {
    if (!d_omega || !d_swap || !d_state || !d_chi) return fail(PFFRG_EINVAL, "null pointer");
    if (n_freq < 2 || n_pairs < 1) return fail(PFFRG_EINVAL, "need n_freq >= 2 and n_pairs >= 1");
    if (n_freq > PFFRG_NOALLOC_MAX_FREQ || n_pairs > PFFRG_NOALLOC_MAX_PAIRS)
        return fail(PFFRG_EUNSUPPORTED, "pffrg_chi_noalloc: more than " + std::to_string(PFFRG_NOALLOC_MAX_FREQ) +
                                            " frequencies or " + std::to_string(PFFRG_NOALLOC_MAX_PAIRS) +
                                            " pairs (the size of its fixed scratch area)");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(PFFRG_EINVAL, "lambda must be finite and > 0");
    double* s = nullptr;
    TRY(scratch_address(&s));
    double* cw = s + kOffCw;
    double* cq = s + kOffCq;
    double* cg2 = s + kOffCg2;
    int* cn = reinterpret_cast<int*>(s + kOffCn);
    double* part = s + kOffPart;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_chi_nodes, dim3(1), dim3(64), 0, st, d_omega, n_freq, lambda, d_state, cw, cq, cg2, cn);
    TRY(launch_check("k_chi_nodes"));
    hipLaunchKernelGGL(k_chi_pairs, dim3(n_pairs, kChiSlices), dim3(kChiThreads), 0, st, d_omega, n_freq, n_pairs,
                       d_swap, d_state, (const double*)cw, (const double*)cq, (const double*)cg2, (const int*)cn,
                       part);
    TRY(launch_check("k_chi_pairs"));
    hipLaunchKernelGGL(k_chi_final, dim3(1), dim3(64), 0, st, n_pairs, (const double*)cq, (const double*)cg2,
                       (const int*)cn, (const double*)part, d_chi);
    return launch_check("k_chi_final");
}

}  // extern "C"
