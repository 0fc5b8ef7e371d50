// pffrg.hip -- host side of the C ABI declared in include/pffrg.h.
//
// A context owns device copies of the lattice and mesh tables and every
// scratch buffer, all allocated in pffrg_create.  The flow kernels live in
// kernels_flow.h, correlations and Runge-Kutta vector kernels in
// kernels_obs.h.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pffrg.h"
#include "host_common.h"
#include "kernels_flow.h"
#include "kernels_obs.h"
#include "kernels_adj.h"
#include "kernels_xyz.h"
#include "kernels_tri.h"

using namespace pffrg;
using namespace pffrg_host;

namespace {

constexpr int kNumK = 7;     // Dormand-Prince stages (RK4 uses the first three)
constexpr int kRedBlocks = 512;

}  // namespace

struct pffrg_ctx {
    int nf = 0, ns = 0, nq = 0, nsu = 0;
    int nc = 2;                     // vertex strains: 2 (SU(2)), 4 (XYZ) or 16 (TRI)
    double* coupling3 = nullptr;    // XYZ: [3][ns] couplings Jx, Jy, Jz
    double* coupling9 = nullptr;    // TRI: [ns][3][3] coupling matrices
    int n_rot = 0;                  // TRI spin rotations (0: none; then no swap copy)
    int *rot16 = nullptr, *rpa_rot = nullptr, *swap_rot = nullptr, *site_rot = nullptr;
    int *t_run = nullptr, *t_run_off = nullptr, t_nrun = 0;   // lattice-sum term runs (term_runs)
    long vsz = 0, size = 0;
    pffrg_precision prec = PFFRG_FP64;
    hipStream_t stream = nullptr;
    int device = 0;

    // tables
    double* w = nullptr;
    unsigned char* lut = nullptr;   // [kLutMax] mesh look-up table
    int lut_shift = 0, lut_kmin = 0;
    int *swap = nullptr, *mult = nullptr, *rpa_off = nullptr, *rpa_ka = nullptr,
        *rpa_kb = nullptr, *rpa_cnt = nullptr, *su_a = nullptr, *su_c = nullptr, *uo_a = nullptr,
        *uo_c = nullptr;
    double* coupling = nullptr;
    int nb = 0, nterm = 0;          // chi(k) terms: (basis, site) pairs in range
    int* chi_pair = nullptr;        // [nterm]
    int* site_pair = nullptr;       // [nb * n_sites_total]: reduced pair of (basis site, site), -1 past the range
    int n_sites_total = 0;
    int* rpa_term = nullptr;        // packed lattice-sum terms
    int n_terms = 0;
    double* chi_dr = nullptr;       // [nterm*3]  r_b - r_j

    // scratch
    int* tab_n = nullptr;
    double *tab_w = nullptr, *tab_g = nullptr, *dsig = nullptr;
    void* gv = nullptr;             // packed (Gs, Gd) copy of the state's vertex:
                                    // double2, or float2 in FP32 mode
    double* k[kNumK] = {};
    double *ybuf = nullptr, *ebuf = nullptr;
    double *part_u = nullptr, *part_t = nullptr;   // u- and t-channel parts of one vertex RHS (state layout)
    // how the three channels are launched (pffrg_set_vertex_mode); the
    // concurrent mode runs the s and u channels on `side`, forked from and
    // joined to the context's stream through the two events
    int vertex_mode = PFFRG_VERTEX_AUTO;
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    double *cw = nullptr, *cq = nullptr, *cg2 = nullptr;
    int* cn = nullptr;
    double* chi = nullptr;          // [2*ns]
    double* chi_part = nullptr;     // [ns * kChiSlices * 2] partial double integrals
    double* part = nullptr;         // [2*kRedBlocks]
    double* red = nullptr;          // [2]
    double* host_red = nullptr;     // pinned [2]

    // reverse mode
    int *rpat_off = nullptr, *rpat_ent = nullptr;   // lattice-sum terms grouped by (ka, kb)
    double* ctg = nullptr;          // [3*nf*nq] cotangent of the node weights
    double* cdsig = nullptr;        // [nf] cotangent of d sig / d Lambda
    double* cot_g2 = nullptr;       // [nq] cotangent of g^2 at the correlation nodes
    double* cchi = nullptr;         // [2*ns]
    double* cot_copies = nullptr;   // [kCotCopies * 2 * vsz] spread vertex cotangents

    std::vector<void*> allocs;

    // kernel timing: event pairs recorded around the launches of the kernels
    // whose bit (1 << kernel id) is set
    // position of the last accepted flow step (pffrg_flow_position)
    bool flow_pos = false;
    double flow_lambda = 0.0, flow_log_lambda = 0.0;
    int flow_ladder = 0;

    unsigned prof_mask = 0;
    std::vector<hipEvent_t> ev[PFFRG_K_COUNT];
    int ev_used[PFFRG_K_COUNT] = {};

    FlowArgs args() const {
        FlowArgs A;
        A.w = w; A.nf = nf; A.ns = ns; A.nq = nq;
        A.swap = swap; A.mult = mult; A.rpa_off = rpa_off; A.rpa_ka = rpa_ka;
        A.rpa_kb = rpa_kb; A.rpa_cnt = rpa_cnt; A.su_a = su_a; A.su_c = su_c;
        A.rpa_term = rpa_term; A.n_terms = n_terms;
        A.tab_n = tab_n; A.tab_w = tab_w; A.tab_g = tab_g;
        A.lut = lut; A.lut_shift = lut_shift; A.lut_kmin = lut_kmin;
        A.run = reinterpret_cast<const int2*>(t_run); A.run_off = t_run_off;
        return A;
    }
};

namespace {

template <class T>
pffrg_status dev_alloc(pffrg_ctx* c, T** p, size_t n) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, n * sizeof(T) > 0 ? n * sizeof(T) : 8);
    if (e != hipSuccess) return fail(PFFRG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    c->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return PFFRG_OK;
}

template <class T>
pffrg_status upload(pffrg_ctx* c, T** p, const T* src, size_t n) {
    TRY(dev_alloc(c, p, n));
    if (n) HIP_TRY(hipMemcpy(*p, src, n * sizeof(T), hipMemcpyHostToDevice));
    return PFFRG_OK;
}

void release(pffrg_ctx* c) {
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->join) (void)hipEventDestroy(c->join);
    if (c->side) (void)hipStreamDestroy(c->side);
    c->fork = c->join = nullptr;
    c->side = nullptr;
    for (auto& v : c->ev)
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
    if (c->host_red) (void)hipHostFree(c->host_red);
    c->host_red = nullptr;
}

pffrg_status check_ctx(const pffrg_ctx* c) {
    if (!c) return fail(PFFRG_EINVAL, "null context");
    return PFFRG_OK;
}

// Kernel timing.  Event pairs per kernel id, created on first use; timing
// only (read after a stream synchronisation), so without the system-scope
// fence, whose cache writeback would stall the stream.
constexpr int kMaxTimed = 65536;

bool prof_events(pffrg_ctx* c, int id, int slot) {
    auto& v = c->ev[id];
    while ((int)v.size() <= slot) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) { c->prof_mask = 0; return false; }
        v.push_back(e);
    }
    return true;
}

// Events recorded on the stream before/after the launches of kernel `id`
// (the whole vertex right-hand side, which spans several launches).
void prof_mark(pffrg_ctx* c, int id, bool after) {
    if (!((c->prof_mask >> id) & 1u) || c->ev_used[id] >= kMaxTimed) return;
    const int slot = 2 * c->ev_used[id] + (after ? 1 : 0);
    if (!prof_events(c, id, slot)) return;
    (void)hipEventRecord(c->ev[id][slot], c->stream);
    if (after) ++c->ev_used[id];
}

// The start/stop pair for the next launch of kernel `id` (nulls when it is
// not timed).  The pair is handed to hipExtLaunchKernelGGL, which stamps it
// with the launch's own start and end, so timing adds no packets (and no
// gaps) to the stream.
struct ProfPair {
    hipEvent_t start = nullptr, stop = nullptr;
};

ProfPair prof_pair(pffrg_ctx* c, int id) {
    ProfPair e;
    if (!((c->prof_mask >> id) & 1u) || c->ev_used[id] >= kMaxTimed) return e;
    const int slot = 2 * c->ev_used[id];
    if (!prof_events(c, id, slot + 1)) return e;
    e.start = c->ev[id][slot];
    e.stop = c->ev[id][slot + 1];
    ++c->ev_used[id];
    return e;
}

// LDS of the t-channel launch (shared tables + 4 waves) for ns pairs.
template <class R>
size_t t_lds_bytes(int nf, int ns, int n_terms) {
    const WaveLds<R> L{ns, t_sub((ns + 3) & ~3)};
    return SharedLds{nf, ns, n_terms}.bytes(true) + kWavesPerBlock * L.bytes();
}

size_t t_lds_bytes(int nf, int ns, int n_terms, pffrg_precision prec) {
    return prec == PFFRG_FP32 ? t_lds_bytes<float>(nf, ns, n_terms) : t_lds_bytes<double>(nf, ns, n_terms);
}

// ------------------------------------------------------------ one RHS ---

pffrg_status sigma_rhs(pffrg_ctx* c, double lam, const double* x, double* dsig) {
    FlowArgs A = c->args();
    const ProfPair e = prof_pair(c, PFFRG_K_SIGMA);
    hipExtLaunchKernelGGL(k_sigma_rhs, dim3(c->nf), dim3(kWave), 0, c->stream, e.start, e.stop, 0, A, lam, x,
                          (long)c->vsz, dsig);
    return launch_check("k_sigma_rhs");
}

// Node tables and the packed vertex (c->gv) in precision R, one launch.
template <class R>
pffrg_status tables_pack(pffrg_ctx* c, double lam, const double* x, const double* dsig) {
    const ProfPair e = prof_pair(c, PFFRG_K_TABLES);
    const long packs = (c->vsz + kWave * kPackPerLane - 1) / (kWave * kPackPerLane);
    hipExtLaunchKernelGGL((k_tables_pack<R>), dim3((unsigned)(3 * c->nf + packs)), dim3(kWave), 0, c->stream, e.start,
                          e.stop, 0, c->args(), lam, x, dsig, (long)c->vsz, static_cast<V2<R>*>(c->gv));
    return launch_check("k_tables_pack");
}

// How the channels of one vertex right-hand side run (mode = the context's
// setting; PFFRG_VERTEX_AUTO resolved by the pair count): while a single
// channel is timed they always run as three launches.
int vertex_mode_for(const pffrg_ctx* c) {
    constexpr unsigned kPerChannel = (1u << PFFRG_K_VERTEX_S) | (1u << PFFRG_K_VERTEX_U) | (1u << PFFRG_K_VERTEX_T);
    if (c->prof_mask & kPerChannel) return PFFRG_VERTEX_SEPARATE;
    if (c->vertex_mode != PFFRG_VERTEX_AUTO) return c->vertex_mode;
    // up to 20 pairs one launch, whose s/u and t workgroups share every CU;
    // beyond, the t role's lattice-sum tiles would hold that kernel at 3 waves
    // per SIMD for all three roles, and s+u beside a concurrent t launch,
    // each at its own occupancy, is faster
    return c->ns > 20 ? PFFRG_VERTEX_CONCURRENT : PFFRG_VERTEX_ONE_LAUNCH;
}

template <class R>
pffrg_status launch_vertex_t(pffrg_ctx* c, hipStream_t st, ProfPair e, const FlowArgs& A, int T, double* out,
                             int add) {
    const int blocks = (T + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per = (blocks + 7) / 8;
    const size_t lds_t = t_lds_bytes<R>(c->nf, c->ns, c->n_terms);
    const V2<R>* gv = static_cast<const V2<R>*>(c->gv);
    switch ((c->ns + 3) / 4) {
#define PFFRG_T_CASE(K) \
        case K: hipExtLaunchKernelGGL((k_vertex_t<4 * K, R>), dim3(8 * per), dim3(kWave * kWavesPerBlock), lds_t, st, \
                                      e.start, e.stop, 0, A, gv, T, out, add); break;
        PFFRG_T_CASE(1) PFFRG_T_CASE(2) PFFRG_T_CASE(3) PFFRG_T_CASE(4)
        PFFRG_T_CASE(5) PFFRG_T_CASE(6) PFFRG_T_CASE(7) PFFRG_T_CASE(8)
#undef PFFRG_T_CASE
        default: return fail(PFFRG_EUNSUPPORTED, "pair count out of range");
    }
    return launch_check("k_vertex_t");
}

// The vertex right-hand side in precision R from the packed vertex in c->gv,
// in one of three launch forms with the same sums in the same order,
// dGamma = (s part + u part) + t part, bitwise equal:
//   one launch     k_vertex_stu writes the three parts (s into dx), then
//                  k_sum_channels adds them;
//   separate       s writes dx, u adds, t adds (three launches in turn);
//   concurrent     t writes its part on the context's stream while s writes
//                  dx and u adds on the side stream; after the join the t
//                  part is added.
template <class R>
pffrg_status vertex_rhs(pffrg_ctx* c, double* dx) {
    FlowArgs A = c->args();
    V2<R>* gv = static_cast<V2<R>*>(c->gv);
    const int T = c->nsu * c->nf;
    const int blocks = (T + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per = (blocks + 7) / 8;
    const SharedLds S{c->nf, c->ns, c->n_terms};
    const WaveLds<R> Lsu{c->ns};
    const size_t lds_su = S.bytes(false) + kWavesPerBlock * Lsu.su_bytes();
    const dim3 grid(8 * per), block(kWave * kWavesPerBlock);
    const size_t lds_t = t_lds_bytes<R>(c->nf, c->ns, c->n_terms);
    const long nv = 2L * T * c->ns;
    prof_mark(c, PFFRG_K_VERTEX, false);
    const int mode = vertex_mode_for(c);
    if (mode == PFFRG_VERTEX_ONE_LAUNCH) {
        const size_t lds = lds_t > lds_su ? lds_t : lds_su;
        const ProfPair e = prof_pair(c, PFFRG_K_VERTEX_STU);
        switch ((c->ns + 3) / 4) {
#define PFFRG_STU_CASE(K) \
            case K: hipExtLaunchKernelGGL((k_vertex_stu<4 * K, R>), dim3(24 * per), block, lds, c->stream, e.start, \
                                          e.stop, 0, A, (const V2<R>*)gv, (const int*)c->uo_a, (const int*)c->uo_c, \
                                          T, dx, c->part_u, c->part_t); break;
            PFFRG_STU_CASE(1) PFFRG_STU_CASE(2) PFFRG_STU_CASE(3) PFFRG_STU_CASE(4)
            PFFRG_STU_CASE(5) PFFRG_STU_CASE(6) PFFRG_STU_CASE(7) PFFRG_STU_CASE(8)
#undef PFFRG_STU_CASE
            default: return fail(PFFRG_EUNSUPPORTED, "pair count out of range");
        }
        TRY(launch_check("k_vertex_stu"));
        hipLaunchKernelGGL(k_sum_channels, dim3(grid_for(nv, 256)), dim3(256), 0, c->stream, nv, dx + c->nf,
                           (const double*)c->part_u + c->nf, (const double*)c->part_t + c->nf);
        prof_mark(c, PFFRG_K_VERTEX, true);
        return launch_check("k_sum_channels");
    }
    // concurrent: the t launch goes straight onto the context's stream and
    // the s and u launches onto the side stream behind the fork, so the t
    // workgroups (the larger ones) take the compute units first and the s/u
    // workgroups fill what they leave; the other way round the s/u
    // workgroups refill every slot they free and t waits for their end
    hipStream_t su_stream = c->stream;
    if (mode == PFFRG_VERTEX_CONCURRENT) {
        HIP_TRY(hipEventRecord(c->fork, c->stream));
        HIP_TRY(hipStreamWaitEvent(c->side, c->fork, 0));
        TRY(launch_vertex_t<R>(c, c->stream, ProfPair{}, A, T, c->part_t, 0));
        su_stream = c->side;
    }
    const ProfPair es = prof_pair(c, PFFRG_K_VERTEX_S);
    hipExtLaunchKernelGGL((k_vertex_su<0, R>), grid, block, lds_su, su_stream, es.start, es.stop, 0, A,
                          (const V2<R>*)gv, (const int*)c->uo_a, (const int*)c->uo_c, T, dx);
    const ProfPair eu = prof_pair(c, PFFRG_K_VERTEX_U);
    hipExtLaunchKernelGGL((k_vertex_su<2, R>), grid, block, lds_su, su_stream, eu.start, eu.stop, 0, A,
                          (const V2<R>*)gv, (const int*)c->uo_a, (const int*)c->uo_c, T, dx);
    TRY(launch_check("k_vertex_su"));
    if (mode == PFFRG_VERTEX_CONCURRENT) {
        HIP_TRY(hipEventRecord(c->join, c->side));
        HIP_TRY(hipStreamWaitEvent(c->stream, c->join, 0));
        hipLaunchKernelGGL(k_axpy, dim3(grid_for(nv, 256)), dim3(256), 0, c->stream, nv, 1.0,
                           (const double*)c->part_t + c->nf, dx + c->nf);
        prof_mark(c, PFFRG_K_VERTEX, true);
        return launch_check("k_axpy");
    }
    TRY(launch_vertex_t<R>(c, c->stream, prof_pair(c, PFFRG_K_VERTEX_T), A, T, dx, 1));
    prof_mark(c, PFFRG_K_VERTEX, true);
    return PFFRG_OK;
}

// XYZ right-hand side (kernels_xyz.h): self-energy flow, node tables, the
// packed (x, y, z, d) vertex, then the s (writes), u and t (add) launches.
pffrg_status xyz_sigma_rhs(pffrg_ctx* c, double lam, const double* x, double* dsig) {
    const ProfPair e = prof_pair(c, PFFRG_K_SIGMA);
    hipExtLaunchKernelGGL(k_xyz_sigma, dim3(c->nf), dim3(kWave), 0, c->stream, e.start, e.stop, 0, c->args(), lam, x,
                          (long)c->vsz, dsig);
    return launch_check("k_xyz_sigma");
}

// The XYZ t-channel launch on stream st: adds to dx (add = 1) or writes
// its part (add = 0).
template <class R>
pffrg_status xyz_vertex_t(pffrg_ctx* c, const FlowArgs& A, V4<R>* gv, int T, hipStream_t st, double* dx, int add) {
    const SharedLds S{c->nf, c->ns, c->n_terms};
    const dim3 block(kWave * kWavesPerBlock);
    if (c->ns > kXyzMaxPairs) {
        // four waves per triple, one triple per workgroup (up to 16 pairs the
        // one-wave kernel below is the faster: 0.414 against 0.457 ms per
        // right-hand side at honeycomb range 6 in FP64)
        const int per4 = (T + 7) / 8;
        hipLaunchKernelGGL((k_xyz_t4<2, R>), dim3(8 * per4), block, S.bytes(true) + XyzT4Lds<R>::bytes(), st, A,
                           (const V4<R>*)gv, T, dx, add);
        return launch_check("k_xyz_t4");
    }
    const int blocks = (T + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per = (blocks + 7) / 8;
    hipLaunchKernelGGL(k_xyz_t<R>, dim3(8 * per), block, S.bytes(true) + kWavesPerBlock * XyzWaveLds<R>::bytes(), st,
                       A, (const V4<R>*)gv, T, dx, add);
    return launch_check("k_xyz_t");
}

// The vertex kernels of the XYZ right-hand side in precision R (the packed
// vertex, s writes, u and t add; beyond 16 pairs, in the concurrent mode, t
// beside s and u).
template <class R>
pffrg_status xyz_vertex(pffrg_ctx* c, const FlowArgs& A, const double* x, double* dx) {
    V4<R>* gv = static_cast<V4<R>*>(c->gv);
    hipLaunchKernelGGL(k_xyz_pack<R>, dim3(grid_for(c->vsz, 256)), dim3(256), 0, c->stream, (long)c->vsz,
                       x + c->nf, gv);
    TRY(launch_check("k_xyz_pack"));
    const int T = c->nsu * c->nf;
    const int blocks = (T + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per = (blocks + 7) / 8;
    const SharedLds S{c->nf, c->ns, c->n_terms};
    const size_t lds_su = S.bytes(false) + kWavesPerBlock * XyzWaveLds<R>::bytes();
    const dim3 grid(8 * per), block(kWave * kWavesPerBlock);
    prof_mark(c, PFFRG_K_VERTEX, false);
    // beyond 16 pairs (the four-wave t kernel) the t channel writes its part
    // on the context's stream while s and u run on the side stream, as in
    // the concurrent SU(2) form: (s + u) + t, the order of the launches in
    // turn, so the same bits
    const bool conc = c->ns > kXyzMaxPairs && vertex_mode_for(c) == PFFRG_VERTEX_CONCURRENT;
    hipStream_t su_stream = c->stream;
    if (conc) {
        HIP_TRY(hipEventRecord(c->fork, c->stream));
        HIP_TRY(hipStreamWaitEvent(c->side, c->fork, 0));
        TRY(xyz_vertex_t<R>(c, A, gv, T, c->stream, c->part_t, 0));
        su_stream = c->side;
    }
    hipLaunchKernelGGL((k_xyz_su<0, R>), grid, block, lds_su, su_stream, A, (const V4<R>*)gv, (const int*)c->uo_a,
                       (const int*)c->uo_c, T, dx);
    hipLaunchKernelGGL((k_xyz_su<2, R>), grid, block, lds_su, su_stream, A, (const V4<R>*)gv, (const int*)c->uo_a,
                       (const int*)c->uo_c, T, dx);
    TRY(launch_check("k_xyz_su"));
    if (conc) {
        HIP_TRY(hipEventRecord(c->join, c->side));
        HIP_TRY(hipStreamWaitEvent(c->stream, c->join, 0));
        const long nv = 4L * c->vsz;
        hipLaunchKernelGGL(k_axpy, dim3(grid_for(nv, 256)), dim3(256), 0, c->stream, nv, 1.0,
                           (const double*)c->part_t + c->nf, dx + c->nf);
        prof_mark(c, PFFRG_K_VERTEX, true);
        return launch_check("k_axpy");
    }
    TRY(xyz_vertex_t<R>(c, A, gv, T, c->stream, dx, 1));
    prof_mark(c, PFFRG_K_VERTEX, true);
    return PFFRG_OK;
}

pffrg_status xyz_rhs(pffrg_ctx* c, double lam, const double* x, double* dx) {
    FlowArgs A = c->args();
    TRY(xyz_sigma_rhs(c, lam, x, dx));             // the sigma part of dx is dsig
    const ProfPair et = prof_pair(c, PFFRG_K_TABLES);
    hipExtLaunchKernelGGL(k_node_tables, dim3(3 * c->nf), dim3(kWave), 0, c->stream, et.start, et.stop, 0, A, lam, x,
                          (const double*)dx);
    TRY(launch_check("k_node_tables"));
    if (c->prec == PFFRG_FP32) return xyz_vertex<float>(c, A, x, dx);
    return xyz_vertex<double>(c, A, x, dx);
}

// TRI right-hand side (kernels_tri.h): self-energy flow, node tables, the
// packed sixteen-component vertex, then the s (writes), u and t (add)
// launches, all in FP64.
pffrg_status tri_sigma_rhs(pffrg_ctx* c, double lam, const double* x, double* dsig) {
    const ProfPair e = prof_pair(c, PFFRG_K_SIGMA);
    hipExtLaunchKernelGGL(k_tri_sigma, dim3(c->nf), dim3(kWave), 0, c->stream, e.start, e.stop, 0, c->args(), lam, x,
                          (long)c->vsz, dsig);
    return launch_check("k_tri_sigma");
}

size_t tri_lds_su(int nf, int ns, int nterms) { return SharedLds{nf, ns, nterms}.bytes(false) + kTriWaves * TriSuLds::bytes(); }
size_t tri_lds_t(int nf, int ns, int nterms, int n_rot) {
    return SharedLds{nf, ns, nterms}.bytes(true) + TriRotLds{nterms, n_rot}.bytes() + kTriWaves * TriTLds{ns}.bytes();
}

pffrg_status tri_rhs(pffrg_ctx* c, double lam, const double* x, double* dx) {
    FlowArgs A = c->args();
    TRY(tri_sigma_rhs(c, lam, x, dx));             // the sigma part of dx is dsig
    const ProfPair et = prof_pair(c, PFFRG_K_TABLES);
    hipExtLaunchKernelGGL(k_node_tables, dim3(3 * c->nf), dim3(kWave), 0, c->stream, et.start, et.stop, 0, A, lam, x,
                          (const double*)dx);
    TRY(launch_check("k_node_tables"));
    double* gv = static_cast<double*>(c->gv);
    hipLaunchKernelGGL(k_tri_pack, dim3(grid_for(c->vsz, 256)), dim3(256), 0, c->stream, (long)c->vsz, c->ns, x + c->nf,
                       gv);
    TRY(launch_check("k_tri_pack"));
    const int swap_copy = c->n_rot > 0;
    if (swap_copy) {
        hipLaunchKernelGGL(k_tri_pack_swap, dim3(grid_for(c->vsz, 256)), dim3(256), 0, c->stream, (long)c->vsz, c->ns,
                           (const int*)c->swap, (const int*)c->swap_rot, (const int*)c->rot16, gv);
        TRY(launch_check("k_tri_pack_swap"));
    }
    const int T = c->nsu * c->nf;
    const int blocks = (T + kTriWaves - 1) / kTriWaves;
    const int per = (blocks + 7) / 8;
    const dim3 grid(8 * per), block(kWave * kTriWaves);
    prof_mark(c, PFFRG_K_VERTEX, false);
    const size_t lds_su = tri_lds_su(c->nf, c->ns, c->n_terms);
    hipLaunchKernelGGL(k_tri_su<0>, grid, block, lds_su, c->stream, A, (const double*)gv, (const int*)c->uo_a,
                       (const int*)c->uo_c, T, swap_copy, dx);
    hipLaunchKernelGGL(k_tri_su<2>, grid, block, lds_su, c->stream, A, (const double*)gv, (const int*)c->uo_a,
                       (const int*)c->uo_c, T, swap_copy, dx);
    TRY(launch_check("k_tri_su"));
    if (c->n_rot > 1)
        hipLaunchKernelGGL(k_tri_t<true>, grid, block, tri_lds_t(c->nf, c->ns, c->n_terms, c->n_rot), c->stream, A,
                           (const double*)gv, T, swap_copy, (const int*)c->rpa_rot, (const int*)c->rot16, c->n_rot,
                           c->t_run, c->t_run_off, c->t_nrun, dx);
    else
        hipLaunchKernelGGL(k_tri_t<false>, grid, block, tri_lds_t(c->nf, c->ns, c->n_terms, c->n_rot), c->stream, A,
                           (const double*)gv, T, swap_copy, (const int*)c->rpa_rot, (const int*)c->rot16, c->n_rot,
                           c->t_run, c->t_run_off, c->t_nrun, dx);
    prof_mark(c, PFFRG_K_VERTEX, true);
    return launch_check("k_tri_t");
}

pffrg_status rhs(pffrg_ctx* c, double lam, const double* x, double* dx) {
    if (!(lam > 0.0) || !std::isfinite(lam)) return fail(PFFRG_EINVAL, "lambda must be finite and > 0");
    if (c->nc == 4) return xyz_rhs(c, lam, x, dx);
    if (c->nc == 16) return tri_rhs(c, lam, x, dx);
    TRY(sigma_rhs(c, lam, x, dx));                  // the sigma part of dx is dsig
    if (c->prec == PFFRG_FP32) {
        TRY(tables_pack<float>(c, lam, x, dx));
        return vertex_rhs<float>(c, dx);
    }
    TRY(tables_pack<double>(c, lam, x, dx));
    return vertex_rhs<double>(c, dx);
}

// max-norm error / finiteness readback (synchronises the stream)
pffrg_status reduce_err(pffrg_ctx* c, const double* x, const double* y, const double* e, double atol,
                        double rtol, double* err, bool* finite) {
    hipLaunchKernelGGL(k_err_norm, dim3(kRedBlocks), dim3(kRedThreads), 0, c->stream, (long)c->size, x, y, e,
                       atol, rtol, c->part);
    TRY(launch_check("k_err_norm"));
    hipLaunchKernelGGL(k_err_final, dim3(1), dim3(64), 0, c->stream, kRedBlocks, (const double*)c->part, c->red);
    TRY(launch_check("k_err_final"));
    HIP_TRY(hipMemcpyAsync(c->host_red, c->red, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (err) *err = c->host_red[0];
    if (finite) *finite = c->host_red[1] == 0.0;
    return PFFRG_OK;
}

pffrg_status combine(pffrg_ctx* c, const double* x, const double* const* ks, const double* cs, int m,
                     double* y) {
    Combo C{};
    C.m = m;
    for (int j = 0; j < m; ++j) { C.k[j] = ks[j]; C.c[j] = cs[j]; }
    hipLaunchKernelGGL(k_combine, dim3(grid_for(c->size, 256)), dim3(256), 0, c->stream, (long)c->size, x, C, y);
    return launch_check("k_combine");
}

pffrg_status step_euler(pffrg_ctx* c, double l0, double l1, double* x) {
    TRY(rhs(c, l0, x, c->k[0]));
    const double* ks[1] = {c->k[0]};
    const double cs[1] = {l1 - l0};
    return combine(c, x, ks, cs, 1, x);
}

// classical RK4 in Lambda: stages at l0, l0+h/2, l0+h/2, l1
pffrg_status step_rk4(pffrg_ctx* c, double l0, double l1, double* x) {
    const double h = l1 - l0;
    const double lm = l0 + 0.5 * h;
    double* K = c->k[0];
    double* Y = c->k[1];
    double* Acc = c->k[2];
    const long n = c->size;
    const int gb = grid_for(n, 256);
    TRY(rhs(c, l0, x, K));
    hipLaunchKernelGGL(k_rk_stage, dim3(gb), dim3(256), 0, c->stream, n, (const double*)x, (const double*)K,
                       0.5 * h, Y, h / 6.0, Acc, 1);
    TRY(launch_check("k_rk_stage"));
    TRY(rhs(c, lm, Y, K));
    hipLaunchKernelGGL(k_rk_stage, dim3(gb), dim3(256), 0, c->stream, n, (const double*)x, (const double*)K,
                       0.5 * h, Y, h / 3.0, Acc, 0);
    TRY(launch_check("k_rk_stage"));
    TRY(rhs(c, lm, Y, K));
    hipLaunchKernelGGL(k_rk_stage, dim3(gb), dim3(256), 0, c->stream, n, (const double*)x, (const double*)K,
                       h, Y, h / 3.0, Acc, 0);
    TRY(launch_check("k_rk_stage"));
    TRY(rhs(c, l1, Y, K));
    hipLaunchKernelGGL(k_rk_stage, dim3(gb), dim3(256), 0, c->stream, n, (const double*)Acc, (const double*)K,
                       0.0, (double*)nullptr, h / 6.0, x, 1);
    return launch_check("k_rk_stage");
}

// Dormand-Prince 5(4) (Dormand & Prince 1980) in l = ln Lambda: dx/dl = Lambda dx/dLambda.
struct Dopri {
    static constexpr double c[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
    static constexpr double a[7][6] = {
        {0, 0, 0, 0, 0, 0},
        {1.0 / 5, 0, 0, 0, 0, 0},
        {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
        {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
        {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
        {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
        {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
    static constexpr double e[7] = {35.0 / 384 - 5179.0 / 57600, 0.0, 500.0 / 1113 - 7571.0 / 16695,
                                    125.0 / 192 - 393.0 / 640, -2187.0 / 6784 + 92097.0 / 339200,
                                    11.0 / 84 - 187.0 / 2100, -1.0 / 40};
};
constexpr double Dopri::c[7];
constexpr double Dopri::a[7][6];
constexpr double Dopri::e[7];

// One attempted Dormand-Prince step from l0 with signed step dl.  On entry
// k[0] holds dx/dLambda at (exp(l0), x) (first-same-as-last).  Writes the
// candidate to ybuf, the stage derivatives to k[1..6] and returns the error
// norm.  lam_j are the stage cutoffs.
pffrg_status dopri_attempt(pffrg_ctx* c, double l0, double dl, const double* x, double atol, double rtol,
                           double* err, bool* finite, double lam_out[7]) {
    double lam[7];
    for (int j = 0; j < 7; ++j) lam[j] = std::exp(l0 + Dopri::c[j] * dl);
    for (int i = 1; i < 7; ++i) {
        const double* ks[6];
        double cs[6];
        for (int j = 0; j < i; ++j) { ks[j] = c->k[j]; cs[j] = dl * Dopri::a[i][j] * lam[j]; }
        TRY(combine(c, x, ks, cs, i, c->ybuf));
        TRY(rhs(c, lam[i], c->ybuf, c->k[i]));
    }
    // ybuf holds the 5th-order solution (stage 7 input equals it); error vector
    const double* ks[7];
    double cs[7];
    for (int j = 0; j < 7; ++j) { ks[j] = c->k[j]; cs[j] = dl * Dopri::e[j] * lam[j]; }
    Combo C{};
    C.m = 7;
    for (int j = 0; j < 7; ++j) { C.k[j] = ks[j]; C.c[j] = cs[j]; }
    hipLaunchKernelGGL(k_combine, dim3(grid_for(c->size, 256)), dim3(256), 0, c->stream, (long)c->size,
                       (const double*)nullptr, C, c->ebuf);
    TRY(launch_check("k_combine"));
    TRY(reduce_err(c, x, c->ybuf, c->ebuf, atol, rtol, err, finite));
    for (int j = 0; j < 7; ++j) lam_out[j] = lam[j];
    return PFFRG_OK;
}

pffrg_status observe(pffrg_ctx* c, const pffrg_flow_opts* o, double lam, const double* x, pffrg_observer cb,
                     void* user, int* stop) {
    *stop = 0;
    if (!cb) return PFFRG_OK;
    TRY(pffrg_chi(c, lam, x, c->chi));
    const double* dk = nullptr;
    if (o->n_k > 0) {
        TRY(pffrg_chi_k(c, c->chi, o->n_k, o->d_k, o->d_chi_k));
        dk = o->d_chi_k;
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    *stop = cb(lam, c->chi, dk, user);
    return PFFRG_OK;
}

// ------------------------------------------------------- reverse mode ---

pffrg_status fill(pffrg_ctx* c, double* p, long n, double v) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, v, p);
    return launch_check("k_fill");
}

pffrg_status axpy(pffrg_ctx* c, long n, double alpha, const double* a, double* y) {
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, alpha, a, y);
    return launch_check("k_axpy");
}

// out = J^T v for the right-hand side at (lam, x); out and v must not alias x.
pffrg_status rhs_vjp(pffrg_ctx* c, double lam, const double* x, const double* v, double* out) {
    if (!(lam > 0.0) || !std::isfinite(lam)) return fail(PFFRG_EINVAL, "lambda must be finite and > 0");
    FlowArgs A = c->args();
    // forward pieces at (lam, x)
    TRY(sigma_rhs(c, lam, x, c->dsig));
    hipLaunchKernelGGL(k_node_tables, dim3(3 * c->nf), dim3(kWave), 0, c->stream, A, lam, x, (const double*)c->dsig);
    TRY(launch_check("k_node_tables"));
    TRY(fill(c, out, c->size, 0.0));
    TRY(fill(c, c->ctg, 3L * c->nf * c->nq, 0.0));
    TRY(fill(c, c->cdsig, c->nf, 0.0));
    TRY(axpy(c, c->nf, 1.0, v, c->cdsig));
    double* cgs = out + c->nf;
    double* cgd = cgs + c->vsz;
    const long cstride = 2 * c->vsz;
    TRY(fill(c, c->cot_copies, kCotCopies * cstride, 0.0));
    double* kgs = c->cot_copies;
    double* kgd = kgs + c->vsz;
    const int T = c->nsu * c->nf;
    // the packed (Gs, Gd) copy of the vertex the gathers read
    V2<double>* gv = static_cast<V2<double>*>(c->gv);
    hipLaunchKernelGGL(k_pack<double>, dim3(grid_for(c->vsz, 256)), dim3(256), 0, c->stream, (long)c->vsz,
                       x + c->nf, x + c->nf + c->vsz, gv);
    TRY(launch_check("k_pack"));
    {
        const int blocks = (T + kAdjWaves - 1) / kAdjWaves;
        const int per = (blocks + 7) / 8;
        const size_t lds = SharedLds{c->nf, c->ns, c->n_terms}.bytes(false) + kAdjWaves * AdjWaveLds::bytes();
        hipLaunchKernelGGL(k_vertex_vjp_su<0>, dim3(8 * per), dim3(kWave * kAdjWaves), lds, c->stream, A,
                           (const V2<double>*)gv, (const int*)c->uo_a, (const int*)c->uo_c, T, v, kgs, kgd, cstride, c->ctg);
        TRY(launch_check("k_vertex_vjp_su"));
        hipLaunchKernelGGL(k_vertex_vjp_su<2>, dim3(8 * per), dim3(kWave * kAdjWaves), lds, c->stream, A,
                           (const V2<double>*)gv, (const int*)c->uo_a, (const int*)c->uo_c, T, v, kgs, kgd, cstride, c->ctg);
        TRY(launch_check("k_vertex_vjp_su"));
    }
    {
        const int per = (T + 7) / 8;
        const size_t lds = SharedLds{c->nf, c->ns, c->n_terms}.bytes(false) + AdjTLds{c->ns}.bytes();
        hipLaunchKernelGGL(k_vertex_vjp_t, dim3(8 * per), dim3(kWave), lds, c->stream, A, (const V2<double>*)gv, T,
                           (const int*)c->rpat_off, (const int*)c->rpat_ent, v, kgs, kgd, cstride, c->ctg);
        TRY(launch_check("k_vertex_vjp_t"));
    }
    hipLaunchKernelGGL(k_sum_copies, dim3(grid_for(cstride, 256)), dim3(256), 0, c->stream, cstride, cstride,
                       (const double*)c->cot_copies, cgs);
    TRY(launch_check("k_sum_copies"));
    hipLaunchKernelGGL(k_tables_vjp, dim3(3 * c->nf), dim3(kWave), 0, c->stream, A, lam, x, (const double*)c->dsig,
                       (const double*)c->ctg, out, c->cdsig);
    TRY(launch_check("k_tables_vjp"));
    hipLaunchKernelGGL(k_sigma_vjp, dim3(c->nf), dim3(kWave), 0, c->stream, A, lam, x, (long)c->vsz,
                       (const double*)c->cdsig, cgs, cgd, out);
    return launch_check("k_sigma_vjp");
}

// out = (d chi / d x)^T cchi at (lam, x).
pffrg_status chi_vjp(pffrg_ctx* c, double lam, const double* x, const double* cchi, double* out) {
    hipLaunchKernelGGL(k_chi_nodes, dim3(1), dim3(64), 0, c->stream, (const double*)c->w, c->nf, lam, x, c->cw, c->cq,
                       c->cg2, c->cn);
    TRY(launch_check("k_chi_nodes"));
    TRY(fill(c, out, c->size, 0.0));
    TRY(fill(c, c->cot_g2, c->nq, 0.0));
    hipLaunchKernelGGL(k_chi_pairs_vjp, dim3(c->ns), dim3(kChiThreads), 0, c->stream, (const double*)c->w, c->nf,
                       c->ns, (const int*)c->swap, x, (const double*)c->cw, (const double*)c->cq,
                       (const double*)c->cg2, (const int*)c->cn, cchi, out + c->nf, out + c->nf + c->vsz,
                       c->cot_g2);
    TRY(launch_check("k_chi_pairs_vjp"));
    hipLaunchKernelGGL(k_chi_nodes_vjp, dim3(1), dim3(1), 0, c->stream, (const double*)c->w, c->nf, x,
                       (const double*)c->cw, (const int*)c->cn, (const double*)c->cot_g2, out);
    return launch_check("k_chi_nodes_vjp");
}

}  // namespace

namespace pffrg_host {

pffrg_status check_mesh(const pffrg_mesh* mesh, int max_freq) {
    if (!mesh) return fail(PFFRG_EINVAL, "mesh is null");
    const int nf = mesh->n_freq;
    if (nf < 2 || !mesh->omega) return fail(PFFRG_EINVAL, "mesh needs n_freq >= 2 frequencies");
    for (int i = 0; i < nf; ++i) {
        if (!(mesh->omega[i] > 0.0) || !std::isfinite(mesh->omega[i]))
            return fail(PFFRG_EINVAL, "mesh frequencies must be finite and > 0");
        if (i > 0 && !(mesh->omega[i] > mesh->omega[i - 1]))
            return fail(PFFRG_EINVAL, "mesh must be strictly ascending");
    }
    if (nf > max_freq) return fail(PFFRG_EUNSUPPORTED, "more than 128 frequencies is not supported");
    return PFFRG_OK;
}

pffrg_status check_lattice(const pffrg_lattice* lat, int max_pairs) {
    if (!lat) return fail(PFFRG_EINVAL, "lattice is null");
    const int ns = lat->n_pairs;
    if (ns < 1 || !lat->swap || !lat->mult || !lat->rpa_off || !lat->coupling)
        return fail(PFFRG_EINVAL, "lattice tables incomplete");
    if (ns > max_pairs)
        return fail(PFFRG_EUNSUPPORTED, "more reduced pairs than this kernel build supports (" +
                                            std::to_string(max_pairs) + ")");
    if (lat->swap[0] != 0) return fail(PFFRG_EINVAL, "pair 0 must be the on-site pair (swap[0] == 0)");
    const int nterms = lat->rpa_off[ns];
    if (lat->rpa_off[0] != 0 || nterms < 0) return fail(PFFRG_EINVAL, "bad rpa_off");
    for (int p = 0; p < ns; ++p) {
        if (lat->swap[p] < 0 || lat->swap[p] >= ns) return fail(PFFRG_EINVAL, "swap out of range");
        if (lat->mult[p] < 1) return fail(PFFRG_EINVAL, "mult must be >= 1");
        if (lat->rpa_off[p + 1] < lat->rpa_off[p]) return fail(PFFRG_EINVAL, "rpa_off not ascending");
        if (!std::isfinite(lat->coupling[p])) return fail(PFFRG_EINVAL, "couplings must be finite");
    }
    if (nterms > 0 && (!lat->rpa_ka || !lat->rpa_kb || !lat->rpa_cnt))
        return fail(PFFRG_EINVAL, "lattice-sum terms missing");
    for (int q = 0; q < nterms; ++q) {
        if (lat->rpa_ka[q] < 0 || lat->rpa_ka[q] >= ns || lat->rpa_kb[q] < 0 || lat->rpa_kb[q] >= ns)
            return fail(PFFRG_EINVAL, "rpa term pair out of range");
        if (lat->rpa_cnt[q] < 1 || lat->rpa_cnt[q] > 32767)
            return fail(PFFRG_EINVAL, "rpa_cnt out of range [1, 32767]");
    }
    if (lat->n_basis < 1 || lat->n_sites_total < 1 || !lat->site_pair || !lat->site_pos || !lat->basis_pos)
        return fail(PFFRG_EINVAL, "site map incomplete");
    for (long k = 0; k < (long)lat->n_basis * lat->n_sites_total; ++k)
        if (lat->site_pair[k] < -1 || lat->site_pair[k] >= ns) return fail(PFFRG_EINVAL, "site_pair out of range");
    return PFFRG_OK;
}

}  // namespace pffrg_host

// ====================================================================== ABI

extern "C" {

const char* pffrg_last_error(void) { return g_err.c_str(); }

const char* pffrg_status_string(pffrg_status s) {
    switch (s) {
        case PFFRG_OK: return "PFFRG_OK";
        case PFFRG_EINVAL: return "PFFRG_EINVAL";
        case PFFRG_EHIP: return "PFFRG_EHIP";
        case PFFRG_ENOMEM: return "PFFRG_ENOMEM";
        case PFFRG_EDIVERGED: return "PFFRG_EDIVERGED";
        case PFFRG_EUNSUPPORTED: return "PFFRG_EUNSUPPORTED";
    }
    return "unknown status";
}

}  // extern "C"

namespace {

// The context of pffrg_create (coupling3 and coupling9 NULL, SU(2)),
// pffrg_create_xyz (coupling3 = [3][ns] couplings Jx, Jy, Jz) and
// pffrg_create_tri (coupling9 = [ns][3][3] coupling matrices); lat->coupling
// is read for SU(2) only.
// The 16-component form of spin rotation r (rows as in pffrg_spin_rot):
// word m = 4 mu + nu -> (4 pi(mu) + pi(nu)) | (s(mu) s(nu) < 0) << 4.
void rot16_of(const int* rows, int* out) {
    int pi[4] = {0, 0, 0, 0}, sg[4] = {1, 1, 1, 1};
    for (int a = 0; a < 3; ++a) {
        pi[a + 1] = std::abs(rows[a]);
        sg[a + 1] = rows[a] < 0 ? -1 : 1;
    }
    for (int m = 0; m < 16; ++m) out[m] = (4 * pi[m / 4] + pi[m % 4]) | ((sg[m / 4] * sg[m % 4] < 0) << 4);
}

pffrg_status check_spin_rot(const pffrg_spin_rot* r, const pffrg_lattice* lat) {
    if (r->n_rot < 1 || r->n_rot > 24 || !r->rot || !r->swap_rot || !r->site_rot ||
        (lat->rpa_off[lat->n_pairs] > 0 && (!r->rpa_rot_a || !r->rpa_rot_b)))
        return fail(PFFRG_EINVAL, "spin rotations: bad table");
    for (int i = 0; i < r->n_rot; ++i) {
        const int* w = r->rot + 3 * i;
        bool seen[3] = {false, false, false};
        int m[3][3] = {};
        for (int a = 0; a < 3; ++a) {
            const int v = std::abs(w[a]);
            if (v < 1 || v > 3 || seen[v - 1]) return fail(PFFRG_EINVAL, "spin rotations: a row is not a signed unit vector");
            seen[v - 1] = true;
            m[a][v - 1] = w[a] < 0 ? -1 : 1;
        }
        const int det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                        m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
        if (det != 1) return fail(PFFRG_EINVAL, "spin rotations: det W must be +1");
        if (i == 0 && !(w[0] == 1 && w[1] == 2 && w[2] == 3)) return fail(PFFRG_EINVAL, "spin rotation 0 must be the identity");
    }
    auto in_range = [&](const int* a, long n) {
        for (long i = 0; i < n; ++i)
            if (a[i] < 0 || a[i] >= r->n_rot) return false;
        return true;
    };
    const long nt = lat->rpa_off[lat->n_pairs];
    if (!in_range(r->swap_rot, lat->n_pairs) || !in_range(r->site_rot, (long)lat->n_basis * lat->n_sites_total) ||
        (nt > 0 && (!in_range(r->rpa_rot_a, nt) || !in_range(r->rpa_rot_b, nt))))
        return fail(PFFRG_EINVAL, "spin rotations: id out of range");
    return PFFRG_OK;
}

pffrg_status create_ctx(const pffrg_lattice* lat_in, const double* coupling3, const double* coupling9,
                        const pffrg_spin_rot* srot, const pffrg_mesh* mesh, pffrg_precision prec, void* stream,
                        pffrg_ctx** out) {
    if (!out) return fail(PFFRG_EINVAL, "out is null");
    *out = nullptr;
    if (!lat_in) return fail(PFFRG_EINVAL, "null lattice");
    const bool xyz = coupling3 != nullptr, tri = coupling9 != nullptr;
    pffrg_lattice lat_copy = *lat_in;
    if (xyz) lat_copy.coupling = coupling3;        // the x couplings stand in for the table check
    if (tri) lat_copy.coupling = coupling9;        // so do the first entries of the matrices
    const pffrg_lattice* lat = &lat_copy;
    TRY(check_mesh(mesh, kMaxFreq));
    TRY(check_lattice(lat, tri ? kTriMaxPairs : kMaxPairs));
    if (prec != PFFRG_FP64 && prec != PFFRG_FP32) return fail(PFFRG_EINVAL, "unknown precision");
    if (tri && prec != PFFRG_FP64) return fail(PFFRG_EUNSUPPORTED, "TRI contexts run in FP64 only");
    if (xyz) {
        for (int i = 0; i < 3 * lat->n_pairs; ++i)
            if (!std::isfinite(coupling3[i])) return fail(PFFRG_EINVAL, "couplings must be finite");
    }
    if (tri) {
        for (int i = 0; i < 9 * lat->n_pairs; ++i)
            if (!std::isfinite(coupling9[i])) return fail(PFFRG_EINVAL, "couplings must be finite");
        if (srot) TRY(check_spin_rot(srot, lat));
    }
    const int nf = mesh->n_freq, ns = lat->n_pairs;
    const int nterms = lat->rpa_off[ns];

    pffrg_ctx* c = new (std::nothrow) pffrg_ctx;
    if (!c) return fail(PFFRG_ENOMEM, "host allocation failed");
    c->nf = nf;
    c->ns = ns;
    c->nc = tri ? 16 : (xyz ? 4 : 2);
    c->nq = 2 * nf + 10;
    c->nsu = nf * (nf + 1) / 2;
    c->vsz = (long)c->nsu * nf * ns;
    c->size = nf + c->nc * c->vsz;
    c->prec = prec;
    c->stream = static_cast<hipStream_t>(stream);
    c->nb = lat->n_basis;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return fail(PFFRG_EHIP, "no HIP device"); }

    auto body = [&]() -> pffrg_status {
        TRY(upload(c, &c->w, mesh->omega, (size_t)nf));
        {
            unsigned char lut[kLutMax];
            build_mesh_lut(mesh->omega, nf, lut, c->lut_shift, c->lut_kmin);
            TRY(upload(c, &c->lut, lut, (size_t)kLutMax));
        }
        TRY(upload(c, &c->swap, lat->swap, (size_t)ns));
        TRY(upload(c, &c->mult, lat->mult, (size_t)ns));
        TRY(upload(c, &c->rpa_off, lat->rpa_off, (size_t)ns + 1));
        TRY(upload(c, &c->rpa_ka, lat->rpa_ka, (size_t)nterms));
        TRY(upload(c, &c->rpa_kb, lat->rpa_kb, (size_t)nterms));
        TRY(upload(c, &c->rpa_cnt, lat->rpa_cnt, (size_t)nterms));
        {
            std::vector<int> packed(nterms);
            for (int q = 0; q < nterms; ++q) {
                if (lat->rpa_cnt[q] < 1 || lat->rpa_cnt[q] > 32767)
                    return fail(PFFRG_EINVAL, "rpa_cnt out of range [1, 32767]");
                packed[q] = (lat->rpa_ka[q] * ns + lat->rpa_kb[q]) | (lat->rpa_cnt[q] << 16);
            }
            c->n_terms = nterms;
            TRY(upload(c, &c->rpa_term, packed.data(), packed.size()));
        }
        if (xyz) TRY(upload(c, &c->coupling3, coupling3, (size_t)3 * ns));
        else if (tri) TRY(upload(c, &c->coupling9, coupling9, (size_t)9 * ns));
        {
            std::vector<int> run(2 * kWave), run_off(ns + 1);
            c->t_nrun = term_runs(ns, lat->rpa_off, run.data(), run_off.data());
            TRY(upload(c, &c->t_run, run.data(), run.size()));
            TRY(upload(c, &c->t_run_off, run_off.data(), run_off.size()));
        }
        if (tri && srot) {
            c->n_rot = srot->n_rot;
            std::vector<int> r16(16 * (size_t)c->n_rot), rr(nterms);
            for (int i = 0; i < c->n_rot; ++i) rot16_of(srot->rot + 3 * i, r16.data() + 16 * i);
            for (int q = 0; q < nterms; ++q) rr[q] = srot->rpa_rot_a[q] | (srot->rpa_rot_b[q] << 8);
            TRY(upload(c, &c->rot16, r16.data(), r16.size()));
            if (nterms > 0) TRY(upload(c, &c->rpa_rot, rr.data(), rr.size()));
            TRY(upload(c, &c->swap_rot, srot->swap_rot, (size_t)ns));
            TRY(upload(c, &c->site_rot, srot->site_rot, (size_t)lat->n_basis * lat->n_sites_total));
        }
        else TRY(upload(c, &c->coupling, lat->coupling, (size_t)ns));
        {
            // the same terms grouped by (ka, kb): entry = output pair | count << 16
            std::vector<std::vector<int>> by(ns * ns);
            for (int p = 0; p < ns; ++p)
                for (int q = lat->rpa_off[p]; q < lat->rpa_off[p + 1]; ++q)
                    by[lat->rpa_ka[q] * ns + lat->rpa_kb[q]].push_back(p | (lat->rpa_cnt[q] << 16));
            std::vector<int> off(ns * ns + 1, 0), ent;
            for (int e = 0; e < ns * ns; ++e) {
                ent.insert(ent.end(), by[e].begin(), by[e].end());
                off[e + 1] = (int)ent.size();
            }
            TRY(upload(c, &c->rpat_off, off.data(), off.size()));
            TRY(upload(c, &c->rpat_ent, ent.data(), ent.size()));
        }
        std::vector<int> sa(c->nsu), sc(c->nsu);
        for (int a = 0; a < nf; ++a)
            for (int cc = 0; cc <= a; ++cc) { sa[a * (a + 1) / 2 + cc] = a; sc[a * (a + 1) / 2 + cc] = cc; }
        TRY(upload(c, &c->su_a, sa.data(), sa.size()));
        TRY(upload(c, &c->su_c, sc.data(), sc.size()));
        // the same wedge in u-major order (u-channel launch order)
        std::vector<int> ua, uc;
        for (int cc = 0; cc < nf; ++cc)
            for (int a = cc; a < nf; ++a) { ua.push_back(a); uc.push_back(cc); }
        TRY(upload(c, &c->uo_a, ua.data(), ua.size()));
        TRY(upload(c, &c->uo_c, uc.data(), uc.size()));
        std::vector<int> cp;
        std::vector<double> dr;
        for (int b = 0; b < lat->n_basis; ++b)
            for (int k = 0; k < lat->n_sites_total; ++k) {
                const int pr = lat->site_pair[b * lat->n_sites_total + k];
                if (pr < 0) continue;
                if (pr >= ns) return fail(PFFRG_EINVAL, "site_pair out of range");
                cp.push_back(pr);
                for (int d = 0; d < 3; ++d)
                    dr.push_back(lat->basis_pos[3 * b + d] - lat->site_pos[3 * (b * lat->n_sites_total + k) + d]);
            }
        c->nterm = (int)cp.size();
        TRY(upload(c, &c->chi_pair, cp.data(), cp.size()));
        c->n_sites_total = lat->n_sites_total;
        TRY(upload(c, &c->site_pair, lat->site_pair, (size_t)lat->n_basis * lat->n_sites_total));
        TRY(upload(c, &c->chi_dr, dr.data(), dr.size()));
        TRY(dev_alloc(c, &c->tab_n, (size_t)3 * nf));
        TRY(dev_alloc(c, &c->tab_w, (size_t)3 * nf * c->nq));
        TRY(dev_alloc(c, &c->tab_g, (size_t)3 * nf * c->nq));
        TRY(dev_alloc(c, &c->dsig, (size_t)nf));
        {
            double2* g2 = nullptr;      // large enough for either precision (XYZ: 32 bytes per element, TRI 128;
                                        // TRI with spin rotations twice that: the pre-rotated exchanged pairs)
            TRY(dev_alloc(c, &g2, (size_t)(c->nc / 2) * c->vsz * (c->n_rot > 0 ? 2 : 1)));
            c->gv = g2;
        }
        for (int j = 0; j < kNumK; ++j) TRY(dev_alloc(c, &c->k[j], (size_t)c->size));
        TRY(dev_alloc(c, &c->ybuf, (size_t)c->size));
        TRY(dev_alloc(c, &c->part_u, (size_t)c->size));
        TRY(dev_alloc(c, &c->part_t, (size_t)c->size));
        TRY(dev_alloc(c, &c->ebuf, (size_t)c->size));
        TRY(dev_alloc(c, &c->cw, (size_t)c->nq));
        TRY(dev_alloc(c, &c->cq, (size_t)c->nq));
        TRY(dev_alloc(c, &c->cg2, (size_t)c->nq));
        TRY(dev_alloc(c, &c->cn, 1));
        TRY(dev_alloc(c, &c->chi, (size_t)c->nc * ns));
        TRY(dev_alloc(c, &c->chi_part, (size_t)c->nc * ns * kChiSlices));
        TRY(dev_alloc(c, &c->part, (size_t)2 * kRedBlocks));
        TRY(dev_alloc(c, &c->red, 2));
        TRY(dev_alloc(c, &c->ctg, (size_t)3 * nf * c->nq));
        TRY(dev_alloc(c, &c->cdsig, (size_t)nf));
        TRY(dev_alloc(c, &c->cot_g2, (size_t)c->nq));
        TRY(dev_alloc(c, &c->cchi, (size_t)2 * ns));
        if (c->nc == 2) TRY(dev_alloc(c, &c->cot_copies, (size_t)kCotCopies * 2 * c->vsz));   // reverse mode only
        HIP_TRY(hipHostMalloc((void**)&c->host_red, 2 * sizeof(double), hipHostMallocDefault));
        // second stream (default priority) and fork/join events of the
        // concurrent vertex mode
        HIP_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&c->join, hipEventDisableTiming));
        if (!tri && t_lds_bytes(nf, ns, nterms, prec) > 64 * 1024)
            return fail(PFFRG_EUNSUPPORTED, "vertex kernel LDS budget exceeded");
        if (tri && (tri_lds_su(nf, ns, nterms) > 64 * 1024 || tri_lds_t(nf, ns, nterms, c->n_rot) > 64 * 1024))
            return fail(PFFRG_EUNSUPPORTED, "TRI vertex kernel LDS budget exceeded");
        if (xyz && (SharedLds{nf, ns, nterms}.bytes(true) + kWavesPerBlock * XyzWaveLds<double>::bytes() > 64 * 1024 ||
                    SharedLds{nf, ns, nterms}.bytes(true) + XyzT4Lds<double>::bytes() > 64 * 1024))
            return fail(PFFRG_EUNSUPPORTED, "XYZ vertex kernel LDS budget exceeded");
        return PFFRG_OK;
    };
    pffrg_status st = body();
    if (st != PFFRG_OK) {
        release(c);
        delete c;
        return st;
    }
    *out = c;
    return PFFRG_OK;
}

pffrg_status no_xyz(const pffrg_ctx* c, const char* what) {
    if (c->nc == 4) return fail(PFFRG_EUNSUPPORTED, std::string(what) + " is not available for XYZ contexts");
    if (c->nc == 16) return fail(PFFRG_EUNSUPPORTED, std::string(what) + " is not available for TRI contexts");
    return PFFRG_OK;
}

}  // namespace

extern "C" {

pffrg_status pffrg_create(const pffrg_lattice* lat, const pffrg_mesh* mesh, pffrg_precision prec, void* stream,
                          pffrg_ctx** out) {
    return create_ctx(lat, nullptr, nullptr, nullptr, mesh, prec, stream, out);
}

pffrg_status pffrg_create_xyz(const pffrg_lattice* lat, const double* coupling3, const pffrg_mesh* mesh,
                              pffrg_precision prec, void* stream, pffrg_ctx** out) {
    if (!coupling3) {
        if (out) *out = nullptr;
        return fail(PFFRG_EINVAL, "null XYZ couplings");
    }
    return create_ctx(lat, coupling3, nullptr, nullptr, mesh, prec, stream, out);
}

pffrg_status pffrg_create_tri(const pffrg_lattice* lat, const double* coupling9, const pffrg_spin_rot* srot,
                              const pffrg_mesh* mesh, pffrg_precision prec, void* stream, pffrg_ctx** out) {
    if (!coupling9) {
        if (out) *out = nullptr;
        return fail(PFFRG_EINVAL, "null TRI couplings");
    }
    return create_ctx(lat, nullptr, coupling9, srot, mesh, prec, stream, out);
}

pffrg_status pffrg_destroy(pffrg_ctx* c) {
    if (!c) return PFFRG_OK;
    (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
    return PFFRG_OK;
}

pffrg_status pffrg_set_vertex_mode(pffrg_ctx* c, int mode) {
    TRY(check_ctx(c));
    if (mode < PFFRG_VERTEX_AUTO || mode > PFFRG_VERTEX_CONCURRENT) return fail(PFFRG_EINVAL, "unknown vertex mode");
    c->vertex_mode = mode;
    return PFFRG_OK;
}

pffrg_status pffrg_set_stream(pffrg_ctx* c, void* stream) {
    TRY(check_ctx(c));
    c->stream = static_cast<hipStream_t>(stream);
    return PFFRG_OK;
}

pffrg_status pffrg_state_size(const pffrg_ctx* c, size_t* n) {
    TRY(check_ctx(c));
    if (!n) return fail(PFFRG_EINVAL, "null output");
    *n = (size_t)c->size;
    return PFFRG_OK;
}

pffrg_status pffrg_init_state(pffrg_ctx* c, double* x) {
    TRY(check_ctx(c));
    if (!x) return fail(PFFRG_EINVAL, "null state");
    if (c->nc == 4) {
        hipLaunchKernelGGL(k_xyz_init_state, dim3(grid_for(c->size, 256)), dim3(256), 0, c->stream, (long)c->size,
                           c->nf, c->ns, (const double*)c->coupling3, x);
        return launch_check("k_xyz_init_state");
    }
    if (c->nc == 16) {
        hipLaunchKernelGGL(k_tri_init_state, dim3(grid_for(c->size, 256)), dim3(256), 0, c->stream, (long)c->size,
                           c->nf, c->ns, (const double*)c->coupling9, x);
        return launch_check("k_tri_init_state");
    }
    hipLaunchKernelGGL(k_init_state, dim3(grid_for(c->size, 256)), dim3(256), 0, c->stream, (long)c->size, c->nf,
                       c->ns, (const double*)c->coupling, x);
    return launch_check("k_init_state");
}

pffrg_status pffrg_rhs(pffrg_ctx* c, double lambda, const double* x, double* dx) {
    TRY(check_ctx(c));
    if (!x || !dx) return fail(PFFRG_EINVAL, "null state");
    if (x == dx) return fail(PFFRG_EINVAL, "state and derivative must not overlap");
    return rhs(c, lambda, x, dx);
}

pffrg_status pffrg_sigma_rhs(pffrg_ctx* c, double lambda, const double* x, double* dsig) {
    TRY(check_ctx(c));
    if (!x || !dsig) return fail(PFFRG_EINVAL, "null pointer");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(PFFRG_EINVAL, "lambda must be finite and > 0");
    if (c->nc == 4) return xyz_sigma_rhs(c, lambda, x, dsig);
    if (c->nc == 16) return tri_sigma_rhs(c, lambda, x, dsig);
    return sigma_rhs(c, lambda, x, dsig);
}

pffrg_status pffrg_step(pffrg_ctx* c, pffrg_scheme scheme, double l0, double l1, double* x) {
    TRY(check_ctx(c));
    if (!x) return fail(PFFRG_EINVAL, "null state");
    if (!(l0 > 0.0) || !(l1 > 0.0) || !std::isfinite(l0) || !std::isfinite(l1))
        return fail(PFFRG_EINVAL, "cutoffs must be finite and > 0");
    switch (scheme) {
        case PFFRG_EULER: return step_euler(c, l0, l1, x);
        case PFFRG_RK4: return step_rk4(c, l0, l1, x);
        default: return fail(PFFRG_EINVAL, "pffrg_step takes PFFRG_EULER or PFFRG_RK4");
    }
}

pffrg_status pffrg_chi(pffrg_ctx* c, double lambda, const double* x, double* chi) {
    TRY(check_ctx(c));
    if (!x || !chi) return fail(PFFRG_EINVAL, "null pointer");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(PFFRG_EINVAL, "lambda must be finite and > 0");
    hipLaunchKernelGGL(k_chi_nodes, dim3(1), dim3(64), 0, c->stream, (const double*)c->w, c->nf, lambda, x, c->cw,
                       c->cq, c->cg2, c->cn);
    TRY(launch_check("k_chi_nodes"));
    if (c->nc == 4) {
        hipLaunchKernelGGL(k_xyz_chi_pairs, dim3(c->ns, kChiSlices), dim3(kChiThreads), 0, c->stream,
                           (const double*)c->w, c->nf, c->ns, (const int*)c->swap, x, (const double*)c->cw,
                           (const double*)c->cq, (const double*)c->cg2, (const int*)c->cn, c->chi_part);
        TRY(launch_check("k_xyz_chi_pairs"));
        hipLaunchKernelGGL(k_xyz_chi_final, dim3(1), dim3(64), 0, c->stream, c->ns, (const double*)c->cq,
                           (const double*)c->cg2, (const int*)c->cn, (const double*)c->chi_part, chi);
        return launch_check("k_xyz_chi_final");
    }
    if (c->nc == 16) {
        hipLaunchKernelGGL(k_tri_chi_pairs, dim3(c->ns, kChiSlices), dim3(kChiThreads), 0, c->stream,
                           (const double*)c->w, c->nf, c->ns, (const int*)c->swap, x, (const double*)c->cw,
                           (const double*)c->cq, (const double*)c->cg2, (const int*)c->cn,
                           (const int*)c->swap_rot, (const int*)c->rot16, c->chi_part);
        TRY(launch_check("k_tri_chi_pairs"));
        hipLaunchKernelGGL(k_tri_chi_final, dim3(1), dim3(64), 0, c->stream, c->ns, (const double*)c->cq,
                           (const double*)c->cg2, (const int*)c->cn, (const double*)c->chi_part, chi);
        return launch_check("k_tri_chi_final");
    }
    hipLaunchKernelGGL(k_chi_pairs, dim3(c->ns, kChiSlices), dim3(kChiThreads), 0, c->stream, (const double*)c->w,
                       c->nf, c->ns, (const int*)c->swap, x, (const double*)c->cw, (const double*)c->cq,
                       (const double*)c->cg2, (const int*)c->cn, c->chi_part);
    TRY(launch_check("k_chi_pairs"));
    hipLaunchKernelGGL(k_chi_final, dim3(1), dim3(64), 0, c->stream, c->ns, (const double*)c->cq,
                       (const double*)c->cg2, (const int*)c->cn, (const double*)c->chi_part, chi);
    return launch_check("k_chi_final");
}

pffrg_status pffrg_chi_k(pffrg_ctx* c, const double* chi, int nk, const double* kp, double* out) {
    TRY(check_ctx(c));
    if (nk < 0 || (nk > 0 && (!chi || !kp || !out))) return fail(PFFRG_EINVAL, "bad chi(k) arguments");
    if (nk == 0) return PFFRG_OK;
    // SU(2): 3 chi^zz; XYZ: chi^xx + chi^yy + chi^zz; TRI: chi^{11} + chi^{22} + chi^{33}
    // (components 5, 10 and 15 of the sixteen)
    const double* c0 = c->nc == 16 ? chi + 5 * c->ns : chi;
    const int stride = c->nc == 16 ? 5 * c->ns : c->ns;
    hipLaunchKernelGGL(k_chi_k, dim3((nk + kChiKWaves - 1) / kChiKWaves), dim3(64 * kChiKWaves), 0, c->stream, c->nterm,
                       (const int*)c->chi_pair, (const double*)c->chi_dr, 1.0 / c->nb, c0, c->nc == 2 ? 1 : 3,
                       stride, c->nc == 2 ? 3.0 : 1.0, nk, kp, out);
    return launch_check("k_chi_k");
}

pffrg_status pffrg_chi_sites(pffrg_ctx* c, const double* chi, double* out) {
    TRY(check_ctx(c));
    if (!chi || !out) return fail(PFFRG_EINVAL, "null correlations");
    const int nbs = c->nb * c->n_sites_total;
    if (c->nc == 16 && c->n_rot > 0) {
        hipLaunchKernelGGL(k_tri_chi_sites, dim3(grid_for(16L * nbs, 256)), dim3(256), 0, c->stream, c->ns, nbs,
                           (const int*)c->site_pair, (const int*)c->site_rot, (const int*)c->rot16, chi, out);
        return launch_check("k_tri_chi_sites");
    }
    hipLaunchKernelGGL(k_chi_sites, dim3(grid_for((long)c->nc * nbs, 256)), dim3(256), 0, c->stream, c->nc, c->ns,
                       nbs, (const int*)c->site_pair, chi, out);
    return launch_check("k_chi_sites");
}

pffrg_status pffrg_flow(pffrg_ctx* c, const pffrg_flow_opts* o, double* x, pffrg_observer cb, void* user,
                        int* n_steps) {
    TRY(check_ctx(c));
    if (!o || !x) return fail(PFFRG_EINVAL, "null options or state");
    if (o->n_k < 0 || (o->n_k > 0 && (!o->d_k || !o->d_chi_k))) return fail(PFFRG_EINVAL, "bad k-point arguments");
    int steps = 0;
    if (n_steps) *n_steps = 0;
    c->flow_pos = false;
    if (o->scheme == PFFRG_EULER || o->scheme == PFFRG_RK4) {
        if (o->n_lambda < 2 || !o->lambdas) return fail(PFFRG_EINVAL, "fixed schedule needs >= 2 cutoffs");
        for (int i = 0; i < o->n_lambda; ++i)
            if (!(o->lambdas[i] > 0.0) || !std::isfinite(o->lambdas[i]))
                return fail(PFFRG_EINVAL, "cutoffs must be finite and > 0");
        for (int i = 0; i + 1 < o->n_lambda; ++i) {
            HIP_TRY(hipMemcpyAsync(c->ybuf, x, sizeof(double) * c->size, hipMemcpyDeviceToDevice, c->stream));
            TRY(pffrg_step(c, o->scheme, o->lambdas[i], o->lambdas[i + 1], x));
            bool fin = true;
            TRY(reduce_err(c, nullptr, x, nullptr, 0.0, 0.0, nullptr, &fin));
            if (!fin) {
                HIP_TRY(hipMemcpyAsync(x, c->ybuf, sizeof(double) * c->size, hipMemcpyDeviceToDevice, c->stream));
                HIP_TRY(hipStreamSynchronize(c->stream));
                if (n_steps) *n_steps = steps;
                return fail(PFFRG_EDIVERGED, "state not finite after step to lambda = " +
                                                 std::to_string(o->lambdas[i + 1]));
            }
            ++steps;
            if (n_steps) *n_steps = steps;
            c->flow_pos = true;
            c->flow_lambda = o->lambdas[i + 1];
            c->flow_log_lambda = std::log(o->lambdas[i + 1]);
            c->flow_ladder = i + 1;
            int stop = 0;
            TRY(observe(c, o, o->lambdas[i + 1], x, cb, user, &stop));
            if (stop) break;
        }
        return PFFRG_OK;
    }
    if (o->scheme != PFFRG_DOPRI54) return fail(PFFRG_EINVAL, "unknown scheme");
    const double lend = std::log(o->lam_stop);
    const double lstart = o->resume ? o->resume_log_lambda : std::log(o->lam_start);
    const bool down = o->resume ? lstart > lend : o->lam_start > o->lam_stop;
    if (!down || !(o->lam_stop > 0.0) || !(o->h0 > 0.0) || !(o->hmin > 0.0) || !(o->rtol >= 0.0) ||
        !(o->atol >= 0.0) || !(o->rtol + o->atol > 0.0) || !std::isfinite(lstart))
        return fail(PFFRG_EINVAL, "bad adaptive options");
    double l = lstart;
    // Step sizes live on the ladder h0 * 2^(m/4); the controller only moves
    // the integer m, so the accepted cutoffs are a deterministic function of
    // accept/reject decisions and reproduce across implementations whose
    // error estimates differ by rounding.
    int m = o->resume ? o->resume_ladder : 0;
    auto ladder = [&](int mm) { return o->h0 * std::pow(2.0, mm / 4.0); };
    auto quarter_steps = [](double fac) { return (int)std::lround(4.0 * std::log2(fac)); };
    const int maxs = o->max_steps > 0 ? o->max_steps : 1000000;
    // The sharp cutoff makes the right-hand side jump where Lambda crosses
    // w_n/2 (a propagator's step function at a delta point switches for a
    // transfer frequency w_n = 2 Lambda).  Steps end just above each such
    // breakpoint and the next one restarts just below it.
    std::vector<double> brk;
    {
        std::vector<double> wh(c->nf);
        HIP_TRY(hipMemcpy(wh.data(), c->w, sizeof(double) * c->nf, hipMemcpyDeviceToHost));
        for (double wv : wh) {
            const double lb = std::log(0.5 * wv);
            if (lb < l && lb > lend) brk.push_back(lb);
        }
        std::sort(brk.begin(), brk.end(), [](double a, double b) { return a > b; });
    }
    const double gap = 1e-12;   // in ln Lambda, on each side of a breakpoint
    size_t ib = 0;
    TRY(rhs(c, std::exp(l), x, c->k[0]));
    int attempts = 0;
    while (l > lend) {
        if (++attempts > 50 * maxs) return fail(PFFRG_EDIVERGED, "too many rejected steps");
        while (ib < brk.size() && brk[ib] + gap >= l) ++ib;
        double dl = -ladder(m);
        bool last = false, at_brk = false;
        if (ib < brk.size() && l + dl <= brk[ib] + gap) { dl = (brk[ib] + gap) - l; at_brk = true; }
        if (l + dl <= lend) { dl = lend - l; last = true; at_brk = false; }
        double err = 0.0;
        bool fin = true;
        double lam[7];
        TRY(dopri_attempt(c, l, dl, x, o->atol, o->rtol, &err, &fin, lam));
        if (fin && err <= 1.0) {
            // accept: x <- y, k0 <- k6 (first-same-as-last)
            HIP_TRY(hipMemcpyAsync(x, c->ybuf, sizeof(double) * c->size, hipMemcpyDeviceToDevice, c->stream));
            std::swap(c->k[0], c->k[6]);
            l = last ? lend : l + dl;
            if (at_brk) {
                // jump over the breakpoint; the derivative must be re-evaluated
                l = brk[ib] - gap;
                ++ib;
                TRY(rhs(c, std::exp(l), x, c->k[0]));
            }
            ++steps;
            if (n_steps) *n_steps = steps;
            const double fac = err > 0.0 ? std::fmin(5.0, std::fmax(0.2, 0.9 * std::pow(err, -0.2))) : 5.0;
            const int dm = quarter_steps(fac);
            if (!(at_brk || last) || dm < 0) m += dm;   // a step cut short keeps its size
            c->flow_pos = true;
            c->flow_lambda = std::exp(l);
            c->flow_log_lambda = l;
            c->flow_ladder = m;
            int stop = 0;
            TRY(observe(c, o, std::exp(l), x, cb, user, &stop));
            if (stop || steps >= maxs) break;
        } else {
            const double fac = (fin && err > 0.0) ? std::fmin(1.0, std::fmax(0.2, 0.9 * std::pow(err, -0.2))) : 0.2;
            m += std::min(-1, quarter_steps(fac));
        }
        if (ladder(m) < o->hmin && l > lend)
            return fail(PFFRG_EDIVERGED, "adaptive step fell below hmin at lambda = " + std::to_string(std::exp(l)));
    }
    return PFFRG_OK;
}

pffrg_status pffrg_flow_position(pffrg_ctx* c, double* lambda, double* log_lambda, int* ladder) {
    TRY(check_ctx(c));
    if (!c->flow_pos) return fail(PFFRG_EINVAL, "no accepted flow step on this context");
    if (lambda) *lambda = c->flow_lambda;
    if (log_lambda) *log_lambda = c->flow_log_lambda;
    if (ladder) *ladder = c->flow_ladder;
    return PFFRG_OK;
}

pffrg_status pffrg_init_state_from(pffrg_ctx* c, const double* coupling, double* x) {
    TRY(check_ctx(c));
    TRY(no_xyz(c, "pffrg_init_state_from"));
    if (!x || !coupling) return fail(PFFRG_EINVAL, "null pointer");
    hipLaunchKernelGGL(k_init_state, dim3(grid_for(c->size, 256)), dim3(256), 0, c->stream, (long)c->size, c->nf,
                       c->ns, coupling, x);
    return launch_check("k_init_state");
}

pffrg_status pffrg_rhs_vjp(pffrg_ctx* c, double lambda, const double* x, const double* v, double* out) {
    TRY(check_ctx(c));
    TRY(no_xyz(c, "pffrg_rhs_vjp"));
    if (!x || !v || !out) return fail(PFFRG_EINVAL, "null pointer");
    if (out == x || out == v) return fail(PFFRG_EINVAL, "output must not overlap the inputs");
    return rhs_vjp(c, lambda, x, v, out);
}

pffrg_status pffrg_chi_vjp(pffrg_ctx* c, double lambda, const double* x, const double* cchi, double* out) {
    TRY(check_ctx(c));
    TRY(no_xyz(c, "pffrg_chi_vjp"));
    if (!x || !cchi || !out) return fail(PFFRG_EINVAL, "null pointer");
    if (out == x) return fail(PFFRG_EINVAL, "output must not overlap the state");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(PFFRG_EINVAL, "lambda must be finite and > 0");
    return chi_vjp(c, lambda, x, cchi, out);
}

pffrg_status pffrg_chi_k_vjp(pffrg_ctx* c, const double* ck, int nk, const double* kp, double* cchi) {
    TRY(check_ctx(c));
    TRY(no_xyz(c, "pffrg_chi_k_vjp"));
    if (nk < 0 || !cchi || (nk > 0 && (!ck || !kp))) return fail(PFFRG_EINVAL, "bad chi(k) arguments");
    TRY(fill(c, cchi, 2L * c->ns, 0.0));
    if (nk == 0) return PFFRG_OK;
    hipLaunchKernelGGL(k_chi_k_vjp, dim3((c->nterm + 127) / 128), dim3(128), 0, c->stream, c->nterm,
                       (const int*)c->chi_pair, (const double*)c->chi_dr, 1.0 / c->nb, nk, kp, ck, cchi);
    return launch_check("k_chi_k_vjp");
}

static pffrg_status check_schedule(int n, const double* l) {
    if (n < 2 || !l) return fail(PFFRG_EINVAL, "schedule needs >= 2 cutoffs");
    for (int i = 0; i < n; ++i)
        if (!(l[i] > 0.0) || !std::isfinite(l[i])) return fail(PFFRG_EINVAL, "cutoffs must be finite and > 0");
    return PFFRG_OK;
}

pffrg_status pffrg_flow_checkpoints(pffrg_ctx* c, int n_lambda, const double* lambdas, double* x, double* ckpt) {
    TRY(check_ctx(c));
    TRY(check_schedule(n_lambda, lambdas));
    if (!x || !ckpt) return fail(PFFRG_EINVAL, "null pointer");
    for (int i = 0; i + 1 < n_lambda; ++i) {
        HIP_TRY(hipMemcpyAsync(ckpt + (size_t)i * c->size, x, sizeof(double) * c->size, hipMemcpyDeviceToDevice,
                               c->stream));
        TRY(step_rk4(c, lambdas[i], lambdas[i + 1], x));
    }
    bool fin = true;
    TRY(reduce_err(c, nullptr, x, nullptr, 0.0, 0.0, nullptr, &fin));
    if (!fin) return fail(PFFRG_EDIVERGED, "state not finite at the end of the checkpointed flow");
    return PFFRG_OK;
}

pffrg_status pffrg_flow_vjp(pffrg_ctx* c, int n_lambda, const double* lambdas, const double* ckpt, double* ybar,
                            double* dcoupling) {
    TRY(check_ctx(c));
    TRY(no_xyz(c, "pffrg_flow_vjp"));
    TRY(check_schedule(n_lambda, lambdas));
    if (!ckpt || !ybar) return fail(PFFRG_EINVAL, "null pointer");
    const long n = c->size;
    const int gb = grid_for(n, 256);
    double* K = c->k[0];
    double* Y2 = c->k[1];
    double* Y3 = c->k[2];
    double* Y4 = c->k[3];
    double* Abar = c->k[4];
    double* kbar = c->k[5];
    double* Ybar = c->k[6];
    for (int i = n_lambda - 2; i >= 0; --i) {
        const double* y = ckpt + (size_t)i * n;
        const double l0 = lambdas[i], l1 = lambdas[i + 1];
        const double h = l1 - l0;
        const double lm = l0 + 0.5 * h;
        // the step's stage states, as in step_rk4
        TRY(rhs(c, l0, y, K));
        hipLaunchKernelGGL(k_rk_stage, dim3(gb), dim3(256), 0, c->stream, n, y, (const double*)K, 0.5 * h, Y2, 0.0,
                           (double*)nullptr, 0);
        TRY(launch_check("k_rk_stage"));
        TRY(rhs(c, lm, Y2, K));
        hipLaunchKernelGGL(k_rk_stage, dim3(gb), dim3(256), 0, c->stream, n, y, (const double*)K, 0.5 * h, Y3, 0.0,
                           (double*)nullptr, 0);
        TRY(launch_check("k_rk_stage"));
        TRY(rhs(c, lm, Y3, K));
        hipLaunchKernelGGL(k_rk_stage, dim3(gb), dim3(256), 0, c->stream, n, y, (const double*)K, h, Y4, 0.0,
                           (double*)nullptr, 0);
        TRY(launch_check("k_rk_stage"));
        // reverse: y1 = Acc + (h/6) k4 with Acc = y + (h/6) k1 + (h/3) k2 + (h/3) k3
        HIP_TRY(hipMemcpyAsync(Abar, ybar, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
        const double* ys[4] = {Y4, Y3, Y2, y};
        const double ls[4] = {l1, lm, lm, l0};
        const double cacc[4] = {h / 6.0, h / 3.0, h / 3.0, h / 6.0};   // d y1 / d k_j through Acc (k4: direct)
        const double cy[3] = {h, 0.5 * h, 0.5 * h};                     // d Y_{j+1} / d k_j
        for (int s = 0; s < 4; ++s) {
            TRY(fill(c, kbar, n, 0.0));
            if (s > 0) TRY(axpy(c, n, cy[s - 1], Ybar, kbar));
            TRY(axpy(c, n, cacc[s], Abar, kbar));
            TRY(rhs_vjp(c, ls[s], ys[s], kbar, Ybar));
            TRY(axpy(c, n, 1.0, Ybar, ybar));
        }
    }
    if (dcoupling) {
        hipLaunchKernelGGL(k_coupling_grad, dim3(c->ns), dim3(256), 0, c->stream, (long)c->nsu * c->nf, c->ns,
                           (const double*)(ybar + c->nf), dcoupling);
        TRY(launch_check("k_coupling_grad"));
    }
    return PFFRG_OK;
}

pffrg_status pffrg_set_profiling_mask(pffrg_ctx* c, unsigned mask) {
    TRY(check_ctx(c));
    if (mask >> PFFRG_K_COUNT) return fail(PFFRG_EINVAL, "profiling mask names an unknown kernel");
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->prof_mask = mask;
    for (int i = 0; i < PFFRG_K_COUNT; ++i) c->ev_used[i] = 0;
    return PFFRG_OK;
}

pffrg_status pffrg_set_profiling(pffrg_ctx* c, int on) {
    return pffrg_set_profiling_mask(c, on ? (1u << PFFRG_K_COUNT) - 1u : 0u);
}

pffrg_status pffrg_profile_read(pffrg_ctx* c, int kernel, double* total_ms, int* count) {
    TRY(check_ctx(c));
    if (kernel < 0 || kernel >= PFFRG_K_COUNT || !total_ms || !count) return fail(PFFRG_EINVAL, "bad kernel id");
    HIP_TRY(hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (int i = 0; i < c->ev_used[kernel]; ++i) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[kernel][2 * i], c->ev[kernel][2 * i + 1]));
        tot += ms;
    }
    *total_ms = tot;
    *count = c->ev_used[kernel];
    return PFFRG_OK;
}

}  // extern "C"
