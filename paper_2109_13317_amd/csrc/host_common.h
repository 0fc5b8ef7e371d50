// host_common.h -- error reporting and launch helpers shared by the host
// sources of libpffrg (single flows and batches).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "pffrg.h"

namespace pffrg_host {

// Message of the last failure on this thread (pffrg_last_error).
inline thread_local std::string g_err;

inline pffrg_status fail(pffrg_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return pffrg_host::fail(PFFRG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define TRY(expr)                              \
    do {                                       \
        pffrg_status s_ = (expr);              \
        if (s_ != PFFRG_OK) return s_;         \
    } while (0)

inline pffrg_status launch_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PFFRG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return PFFRG_OK;
}

// Grid of a grid-stride element kernel: enough blocks for n, at most 4096.
inline int grid_for(long n, int threads) {
    long b = (n + threads - 1) / threads;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// Device allocations owned by one object, freed together.
struct DevAllocs {
    std::vector<void*> ptrs;

    template <class T>
    pffrg_status alloc(T** p, size_t n) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, n * sizeof(T) > 0 ? n * sizeof(T) : 8);
        if (e != hipSuccess) return fail(PFFRG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        ptrs.push_back(q);
        *p = static_cast<T*>(q);
        return PFFRG_OK;
    }

    template <class T>
    pffrg_status upload(T** p, const T* src, size_t n) {
        TRY(alloc(p, n));
        if (n) HIP_TRY(hipMemcpy(*p, src, n * sizeof(T), hipMemcpyHostToDevice));
        return PFFRG_OK;
    }

    void release() {
        for (void* q : ptrs) (void)hipFree(q);
        ptrs.clear();
    }
};

// Checks a lattice description against the documented rules of
// pffrg_lattice; `max_pairs` is the kernel build's limit.
pffrg_status check_lattice(const pffrg_lattice* lat, int max_pairs);

// Checks a mesh: n_freq >= 2, finite, > 0, strictly ascending.
pffrg_status check_mesh(const pffrg_mesh* mesh, int max_freq);

}  // namespace pffrg_host
