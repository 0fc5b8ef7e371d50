// pffrg_batch.hip -- host side of the batch entry points of include/pffrg.h:
// many flows on one mesh advanced in lockstep (a phase-diagram scan).
//
// A batch owns concatenated device copies of every point's tables, the
// Runge-Kutta buffers of the whole batch, the tile lists of the persistent
// vertex launch and, once a flow has run, one instantiated hipGraph of an
// RK4 step.  Everything is allocated in pffrg_batch_create.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "pffrg.h"
#include "host_common.h"
#include "kernels_flow.h"
#include "kernels_obs.h"
#include "kernels_batch.h"

using namespace pffrg;
using namespace pffrg_host;

namespace {

constexpr int kMaxSchedule = 65536;   // cutoffs of one batch flow
constexpr int kOrders = 2;            // tile orders the launch can use

// Launch configuration of the persistent vertex kernel.
struct LaunchCfg {
    int per = 64;       // workgroups per XCD
    int order = 0;      // 0: points kept on one XCD, 1: tiles dealt round-robin
    int split = 0;      // 0: one launch for all channels, 1: s+u then t
};

// Tuned configurations, shared by every batch of the process, keyed by
// (frequencies, pair counts, precision).
std::mutex g_tune_mu;
std::map<std::string, LaunchCfg> g_tuned;

std::string tune_key(int nf, const std::vector<int>& ns, pffrg_precision prec) {
    std::vector<int> s(ns);
    std::sort(s.begin(), s.end());
    std::string k = std::to_string(nf) + (prec == PFFRG_FP32 ? "/fp32/" : "/fp64/");
    for (int v : s) k += std::to_string(v) + ",";
    return k;
}

}  // namespace

struct pffrg_batch {
    int np = 0, nf = 0, nq = 0, nsu = 0;
    pffrg_precision prec = PFFRG_FP64;
    hipStream_t stream = nullptr;      // the caller's stream: all work runs here
    hipStream_t cap = nullptr;         // private stream used only to capture the step graph
    std::vector<int> ns, n_terms, nb_chi, chi_off, chi_cnt;
    std::vector<BatchPoint> pts;
    long size = 0, vtot = 0;
    DevAllocs mem;

    double* w = nullptr;
    unsigned char* lut = nullptr;   // [kLutMax] mesh look-up table
    int lut_shift = 0, lut_kmin = 0;
    int *swap = nullptr, *mult = nullptr, *rpa_off = nullptr, *rpa_term = nullptr;
    int *su_a = nullptr, *su_c = nullptr;
    double* coupling = nullptr;
    BatchPoint* d_pts = nullptr;
    int* chi_pair = nullptr;
    double* chi_dr = nullptr;
    double *cw = nullptr, *cq = nullptr, *cg2 = nullptr;
    int* cn = nullptr;
    double* chi_part = nullptr;        // [max ns * kChiSlices * 2]
    int* tab_n = nullptr;
    double *tab_w = nullptr, *tab_g = nullptr;
    void* gv = nullptr;
    double *K = nullptr, *Y = nullptr, *Acc = nullptr;
    double* clk = nullptr;             // [8]: stage cutoffs, h, and a free slot for single calls
    int* step = nullptr;
    double* sched = nullptr;
    double* part = nullptr;
    double* red = nullptr;
    double* host_red = nullptr;

    int2* items[kOrders] = {};
    int* begin[kOrders] = {};
    // the split t launch's lists, per pair class (0: up to 16 pairs, 1: more)
    int2* items_t[2][kOrders] = {};
    int* begin_t[2][kOrders] = {};
    bool has_class[2] = {false, false};
    int shared_bytes = 0, wave_bytes = 0;
    LaunchCfg cfg;
    bool tuned = false;

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const double* graph_x = nullptr;   // the state the instantiated graph advances

    bool profiling = false;
    std::vector<hipEvent_t> ev;
    int ev_used = 0;

    BatchArgs args() const {
        BatchArgs B;
        FlowArgs& A = B.base;
        A.w = w; A.nf = nf; A.ns = ns[0]; A.nq = nq;
        A.swap = swap; A.mult = mult; A.rpa_off = rpa_off; A.rpa_ka = nullptr; A.rpa_kb = nullptr;
        A.rpa_cnt = nullptr; A.rpa_term = rpa_term; A.n_terms = n_terms[0];
        A.su_a = su_a; A.su_c = su_c;
        A.tab_n = tab_n; A.tab_w = tab_w; A.tab_g = tab_g;
        A.lut = lut; A.lut_shift = lut_shift; A.lut_kmin = lut_kmin;
        A.run = nullptr; A.run_off = nullptr;     // batch points have at most 20 pairs
        B.pts = d_pts;
        B.n_points = np;
        return B;
    }
};

namespace {

size_t lds_bytes(const pffrg_batch* b) {
    return (size_t)b->shared_bytes + (size_t)kWavesPerBlock * b->wave_bytes;
}

void drop_graph(pffrg_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_x = nullptr;
}

void release(pffrg_batch* b) {
    drop_graph(b);
    b->mem.release();
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    b->ev.clear();
    if (b->host_red) (void)hipHostFree(b->host_red);
    b->host_red = nullptr;
    if (b->cap) (void)hipStreamDestroy(b->cap);
    b->cap = nullptr;
}

void prof_mark(pffrg_batch* b, hipStream_t s, bool after) {
    if (!b->profiling) return;
    const int slot = 2 * b->ev_used + (after ? 1 : 0);
    if (b->ev_used >= 65536) return;
    while ((int)b->ev.size() <= slot) {
        hipEvent_t e;
        // timing only (read after a stream synchronisation): no system-scope fence
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) { b->profiling = false; return; }
        b->ev.push_back(e);
    }
    (void)hipEventRecord(b->ev[slot], s);
    if (after) ++b->ev_used;
}

// Relative cost of one output triple of a point with ns pairs: the channel
// interpolations and products grow like ns, the lattice-sum matrix like ns^2.
double triple_cost(int ns) { return ns * (142.0 + 4.0 * ns); }

// Tile lists of both orders.  Order 0 assigns whole points to XCDs, largest
// cost first to the least loaded XCD, so each point's vertex is read through
// one L2; order 1 deals all tiles round-robin over the XCDs.
void build_items(const pffrg_batch* b, const std::vector<int>& points, std::vector<int2> out[kOrders],
                 std::vector<int> beg[kOrders]) {
    const int T = b->nsu * b->nf;
    const int tiles = (T + kWavesPerBlock - 1) / kWavesPerBlock;
    std::vector<int> idx(points);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return triple_cost(b->ns[x]) > triple_cost(b->ns[y]); });
    std::vector<double> load(8, 0.0);
    std::vector<std::vector<int>> on(8);
    for (int p : idx) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += triple_cost(b->ns[p]) * T;
        on[x].push_back(p);
    }
    out[0].clear();
    beg[0].assign(9, 0);
    for (int x = 0; x < 8; ++x) {
        beg[0][x] = (int)out[0].size();
        for (int p : on[x])
            for (int t = 0; t < tiles; ++t) out[0].push_back(make_int2(p, t * kWavesPerBlock));
    }
    beg[0][8] = (int)out[0].size();
    std::vector<std::vector<int2>> part(8);
    long k = 0;
    for (int p : points)
        for (int t = 0; t < tiles; ++t, ++k) part[k % 8].push_back(make_int2(p, t * kWavesPerBlock));
    out[1].clear();
    beg[1].assign(9, 0);
    for (int x = 0; x < 8; ++x) {
        beg[1][x] = (int)out[1].size();
        out[1].insert(out[1].end(), part[x].begin(), part[x].end());
    }
    beg[1][8] = (int)out[1].size();
}

// ------------------------------------------------------- one batch RHS --

// dx = d x / d Lambda for every point at the cutoff *lamp (device), on stream s.
template <class R>
pffrg_status batch_rhs_t(pffrg_batch* b, hipStream_t s, const double* lamp, const double* x, double* dx) {
    const BatchArgs B = b->args();
    hipLaunchKernelGGL(k_batch_sigma, dim3(b->nf, b->np), dim3(kWave), 0, s, B, lamp, x, dx);
    TRY(launch_check("k_batch_sigma"));
    hipLaunchKernelGGL(k_batch_tables, dim3(3 * b->nf, b->np), dim3(kWave), 0, s, B, lamp, x, (const double*)dx);
    TRY(launch_check("k_batch_tables"));
    V2<R>* gv = static_cast<V2<R>*>(b->gv);
    const int pb = std::max(1, std::min(64, (int)((b->vtot / b->np + 255) / 256)));
    hipLaunchKernelGGL(k_batch_pack<R>, dim3(pb, b->np), dim3(256), 0, s, B, x, gv);
    TRY(launch_check("k_batch_pack"));
    const LaunchCfg& c = b->cfg;
    const dim3 grid(8 * c.per), block(kWave * kWavesPerBlock);
    const int2* items = b->items[c.order];
    const int* beg = b->begin[c.order];
    prof_mark(b, s, false);
    if (c.split) {
        hipLaunchKernelGGL((k_batch_vertex<R, kSU>), grid, block, lds_bytes(b), s, B, (const V2<R>*)gv, items, beg,
                           b->shared_bytes, b->wave_bytes, dx);
        TRY(launch_check("k_batch_vertex"));
        if (b->has_class[0]) {
            TRY(launch_check("k_batch_vertex"));
            hipLaunchKernelGGL((k_batch_vertex<R, kT, kSmallNsp>), grid, block, lds_bytes(b), s, B, (const V2<R>*)gv,
                               (const int2*)b->items_t[0][c.order], (const int*)b->begin_t[0][c.order],
                               b->shared_bytes, b->wave_bytes, dx);
        }
        if (b->has_class[1]) {
            TRY(launch_check("k_batch_vertex"));
            hipLaunchKernelGGL((k_batch_vertex<R, kT>), grid, block, lds_bytes(b), s, B, (const V2<R>*)gv,
                               (const int2*)b->items_t[1][c.order], (const int*)b->begin_t[1][c.order],
                               b->shared_bytes, b->wave_bytes, dx);
        }
    } else {
        hipLaunchKernelGGL((k_batch_vertex<R, kAll>), grid, block, lds_bytes(b), s, B, (const V2<R>*)gv, items, beg,
                           b->shared_bytes, b->wave_bytes, dx);
    }
    prof_mark(b, s, true);
    return launch_check("k_batch_vertex");
}

pffrg_status batch_rhs(pffrg_batch* b, hipStream_t s, const double* lamp, const double* x, double* dx) {
    return b->prec == PFFRG_FP32 ? batch_rhs_t<float>(b, s, lamp, x, dx) : batch_rhs_t<double>(b, s, lamp, x, dx);
}

// One classical RK4 step of every point, cutoffs from the schedule entry
// *step (device); advances *step.  The same sequence is launched directly
// or captured into the step graph.
pffrg_status rk4_step(pffrg_batch* b, hipStream_t s, double* x) {
    const long n = b->size;
    const int gb = grid_for(n, 256);
    hipLaunchKernelGGL(k_batch_clock, dim3(1), dim3(1), 0, s, (const double*)b->sched, (const int*)b->step, b->clk);
    TRY(launch_check("k_batch_clock"));
    const double am[3] = {0.5, 0.5, 1.0};
    const double bd[3] = {6.0, 3.0, 3.0};
    const double* in = x;
    for (int st = 0; st < 3; ++st) {
        TRY(batch_rhs(b, s, b->clk + st, in, b->K));
        hipLaunchKernelGGL(k_batch_rk_stage, dim3(gb), dim3(256), 0, s, n, (const double*)x, (const double*)b->K,
                           am[st], b->Y, bd[st], b->Acc, st == 0 ? 1 : 0, (const double*)b->clk);
        TRY(launch_check("k_batch_rk_stage"));
        in = b->Y;
    }
    TRY(batch_rhs(b, s, b->clk + 3, b->Y, b->K));
    hipLaunchKernelGGL(k_batch_rk_stage, dim3(gb), dim3(256), 0, s, n, (const double*)b->Acc, (const double*)b->K,
                       0.0, (double*)nullptr, 6.0, x, 1, (const double*)b->clk);
    TRY(launch_check("k_batch_rk_stage"));
    hipLaunchKernelGGL(k_batch_tick, dim3(1), dim3(1), 0, s, b->step);
    return launch_check("k_batch_tick");
}

pffrg_status capture_step(pffrg_batch* b, double* x) {
    drop_graph(b);
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const bool prof = b->profiling;
    b->profiling = false;           // no timing events inside the graph
    pffrg_status st = rk4_step(b, b->cap, x);
    b->profiling = prof;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st != PFFRG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(PFFRG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_x = x;
    return PFFRG_OK;
}

// Per-point finiteness of a batch state: ok[p] = 1 if every value of point p
// is finite.  Synchronises the stream.
pffrg_status finite_points(pffrg_batch* b, const double* x, int* ok) {
    for (int p = 0; p < b->np; ++p) {
        const long off = b->pts[p].x_off;
        const long n = (p + 1 < b->np ? b->pts[p + 1].x_off : b->size) - off;
        hipLaunchKernelGGL(k_err_norm, dim3(64), dim3(kRedThreads), 0, b->stream, n, (const double*)nullptr,
                           x + off, (const double*)nullptr, 0.0, 0.0, b->part);
        TRY(launch_check("k_err_norm"));
        hipLaunchKernelGGL(k_err_final, dim3(1), dim3(64), 0, b->stream, 64, (const double*)b->part, b->red + 2 * p);
        TRY(launch_check("k_err_final"));
    }
    HIP_TRY(hipMemcpyAsync(b->host_red, b->red, sizeof(double) * 2 * b->np, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (int p = 0; p < b->np; ++p) ok[p] = b->host_red[2 * p + 1] == 0.0 ? 1 : 0;
    return PFFRG_OK;
}

pffrg_status check_batch(const pffrg_batch* b) {
    if (!b) return fail(PFFRG_EINVAL, "null batch");
    return PFFRG_OK;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

pffrg_status pffrg_batch_create(int n_points, const pffrg_lattice* const* lats, const pffrg_mesh* mesh,
                                pffrg_precision prec, void* stream, pffrg_batch** out) {
    if (!out) return fail(PFFRG_EINVAL, "out is null");
    *out = nullptr;
    if (n_points < 1 || !lats) return fail(PFFRG_EINVAL, "a batch needs n_points >= 1 lattices");
    if (prec != PFFRG_FP64 && prec != PFFRG_FP32) return fail(PFFRG_EINVAL, "unknown precision");
    TRY(check_mesh(mesh, kMaxFreq));
    for (int p = 0; p < n_points; ++p) {
        pffrg_status st = check_lattice(lats[p], kBatchMaxPairs);
        if (st != PFFRG_OK) return fail(st, "point " + std::to_string(p) + ": " + g_err);
    }
    pffrg_batch* b = new (std::nothrow) pffrg_batch;
    if (!b) return fail(PFFRG_ENOMEM, "host allocation failed");
    const int nf = mesh->n_freq;
    b->np = n_points;
    b->nf = nf;
    b->nq = 2 * nf + 10;
    b->nsu = nf * (nf + 1) / 2;
    b->prec = prec;
    b->stream = static_cast<hipStream_t>(stream);

    auto body = [&]() -> pffrg_status {
        HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        std::vector<int> swap, mult, roff, term, cp;
        std::vector<double> coup, dr;
        long x_off = 0, gv_off = 0;
        int max_shared = 0, max_wave = 0;
        for (int p = 0; p < n_points; ++p) {
            const pffrg_lattice* L = lats[p];
            const int ns = L->n_pairs, nt = L->rpa_off[ns];
            BatchPoint P{};
            P.ns = ns;
            P.n_terms = nt;
            P.pair_off = (int)swap.size();
            P.rpa_off_off = (int)roff.size();
            P.term_off = (int)term.size();
            P.x_off = x_off;
            P.gv_off = gv_off;
            b->pts.push_back(P);
            b->ns.push_back(ns);
            b->n_terms.push_back(nt);
            for (int q = 0; q < ns; ++q) {
                swap.push_back(L->swap[q]);
                mult.push_back(L->mult[q]);
                coup.push_back(L->coupling[q]);
            }
            for (int q = 0; q <= ns; ++q) roff.push_back(L->rpa_off[q]);
            for (int q = 0; q < nt; ++q)
                term.push_back((L->rpa_ka[q] * ns + L->rpa_kb[q]) | (L->rpa_cnt[q] << 16));
            const long v = (long)b->nsu * nf * ns;
            x_off += nf + 2 * v;
            gv_off += v;
            b->chi_off.push_back((int)cp.size());
            for (int bb = 0; bb < L->n_basis; ++bb)
                for (int k = 0; k < L->n_sites_total; ++k) {
                    const int pr = L->site_pair[bb * L->n_sites_total + k];
                    if (pr < 0) continue;
                    cp.push_back(pr);
                    for (int d = 0; d < 3; ++d)
                        dr.push_back(L->basis_pos[3 * bb + d] - L->site_pos[3 * (bb * L->n_sites_total + k) + d]);
                }
            b->chi_cnt.push_back((int)cp.size() - b->chi_off.back());
            b->nb_chi.push_back(L->n_basis);
            max_shared = std::max(max_shared, (int)SharedLds{nf, ns, nt}.bytes(true));
            const int wb = prec == PFFRG_FP32 ? (int)WaveLds<float>{ns, kSub}.all_bytes()
                                              : (int)WaveLds<double>{ns, kSub}.all_bytes();
            max_wave = std::max(max_wave, wb);
        }
        b->size = x_off;
        b->vtot = gv_off;
        b->shared_bytes = (max_shared + 31) & ~31;
        b->wave_bytes = (max_wave + 31) & ~31;
        if (lds_bytes(b) > 64 * 1024) return fail(PFFRG_EUNSUPPORTED, "batch vertex kernel LDS budget exceeded");
        for (const BatchPoint& P : b->pts)
            if ((long)b->nsu * nf * P.ns * 16 > 0x7fffffffL) return fail(PFFRG_EUNSUPPORTED, "point too large");

        TRY(b->mem.upload(&b->w, mesh->omega, (size_t)nf));
        {
            unsigned char lut[kLutMax];
            build_mesh_lut(mesh->omega, nf, lut, b->lut_shift, b->lut_kmin);
            TRY(b->mem.upload(&b->lut, lut, (size_t)kLutMax));
        }
        TRY(b->mem.upload(&b->swap, swap.data(), swap.size()));
        TRY(b->mem.upload(&b->mult, mult.data(), mult.size()));
        TRY(b->mem.upload(&b->rpa_off, roff.data(), roff.size()));
        TRY(b->mem.upload(&b->rpa_term, term.data(), term.size()));
        TRY(b->mem.upload(&b->coupling, coup.data(), coup.size()));
        TRY(b->mem.upload(&b->d_pts, b->pts.data(), b->pts.size()));
        std::vector<int> sa(b->nsu), sc(b->nsu);
        for (int a = 0; a < nf; ++a)
            for (int c = 0; c <= a; ++c) { sa[a * (a + 1) / 2 + c] = a; sc[a * (a + 1) / 2 + c] = c; }
        TRY(b->mem.upload(&b->su_a, sa.data(), sa.size()));
        TRY(b->mem.upload(&b->su_c, sc.data(), sc.size()));
        TRY(b->mem.upload(&b->chi_pair, cp.data(), cp.size()));
        TRY(b->mem.upload(&b->chi_dr, dr.data(), dr.size()));
        TRY(b->mem.alloc(&b->cw, (size_t)b->nq));
        TRY(b->mem.alloc(&b->cq, (size_t)b->nq));
        TRY(b->mem.alloc(&b->cg2, (size_t)b->nq));
        TRY(b->mem.alloc(&b->cn, 1));
        TRY(b->mem.alloc(&b->chi_part, (size_t)2 * kChiSlices * *std::max_element(b->ns.begin(), b->ns.end())));
        TRY(b->mem.alloc(&b->tab_n, (size_t)n_points * 3 * nf));
        TRY(b->mem.alloc(&b->tab_w, (size_t)n_points * 3 * nf * b->nq));
        TRY(b->mem.alloc(&b->tab_g, (size_t)n_points * 3 * nf * b->nq));
        double2* g2 = nullptr;
        TRY(b->mem.alloc(&g2, (size_t)b->vtot));
        b->gv = g2;
        TRY(b->mem.alloc(&b->K, (size_t)b->size));
        TRY(b->mem.alloc(&b->Y, (size_t)b->size));
        TRY(b->mem.alloc(&b->Acc, (size_t)b->size));
        TRY(b->mem.alloc(&b->clk, 8));
        TRY(b->mem.alloc(&b->step, 1));
        TRY(b->mem.alloc(&b->sched, (size_t)kMaxSchedule));
        TRY(b->mem.alloc(&b->part, (size_t)2 * 64));
        TRY(b->mem.alloc(&b->red, (size_t)2 * n_points));
        HIP_TRY(hipHostMalloc((void**)&b->host_red, sizeof(double) * 2 * n_points, hipHostMallocDefault));
        std::vector<int2> items[kOrders];
        std::vector<int> beg[kOrders];
        std::vector<int> all(n_points), cls[2];
        std::iota(all.begin(), all.end(), 0);
        for (int p = 0; p < n_points; ++p) cls[((b->ns[p] + 3) & ~3) > kSmallNsp ? 1 : 0].push_back(p);
        build_items(b, all, items, beg);
        for (int o = 0; o < kOrders; ++o) {
            TRY(b->mem.upload(&b->items[o], items[o].data(), items[o].size()));
            TRY(b->mem.upload(&b->begin[o], beg[o].data(), beg[o].size()));
        }
        for (int k = 0; k < 2; ++k) {
            b->has_class[k] = !cls[k].empty();
            if (!b->has_class[k]) continue;
            build_items(b, cls[k], items, beg);
            for (int o = 0; o < kOrders; ++o) {
                TRY(b->mem.upload(&b->items_t[k][o], items[o].data(), items[o].size()));
                TRY(b->mem.upload(&b->begin_t[k][o], beg[o].data(), beg[o].size()));
            }
        }
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find(tune_key(nf, b->ns, prec));
            if (it != g_tuned.end()) { b->cfg = it->second; b->tuned = true; }
        }
        return PFFRG_OK;
    };
    pffrg_status st = body();
    if (st != PFFRG_OK) {
        release(b);
        delete b;
        return st;
    }
    *out = b;
    return PFFRG_OK;
}

pffrg_status pffrg_batch_destroy(pffrg_batch* b) {
    if (!b) return PFFRG_OK;
    (void)hipStreamSynchronize(b->stream);
    release(b);
    delete b;
    return PFFRG_OK;
}

pffrg_status pffrg_batch_state_offsets(const pffrg_batch* b, size_t* offsets) {
    TRY(check_batch(b));
    if (!offsets) return fail(PFFRG_EINVAL, "null output");
    for (int p = 0; p < b->np; ++p) offsets[p] = (size_t)b->pts[p].x_off;
    offsets[b->np] = (size_t)b->size;
    return PFFRG_OK;
}

pffrg_status pffrg_batch_init_state(pffrg_batch* b, double* x) {
    TRY(check_batch(b));
    if (!x) return fail(PFFRG_EINVAL, "null state");
    for (int p = 0; p < b->np; ++p) {
        const long n = (p + 1 < b->np ? b->pts[p + 1].x_off : b->size) - b->pts[p].x_off;
        hipLaunchKernelGGL(k_init_state, dim3(grid_for(n, 256)), dim3(256), 0, b->stream, n, b->nf, b->ns[p],
                           (const double*)(b->coupling + b->pts[p].pair_off), x + b->pts[p].x_off);
        TRY(launch_check("k_init_state"));
    }
    return PFFRG_OK;
}

pffrg_status pffrg_batch_rhs(pffrg_batch* b, double lambda, const double* x, double* dx) {
    TRY(check_batch(b));
    if (!x || !dx) return fail(PFFRG_EINVAL, "null state");
    if (x == dx) return fail(PFFRG_EINVAL, "state and derivative must not overlap");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(PFFRG_EINVAL, "lambda must be finite and > 0");
    hipLaunchKernelGGL(k_set_value, dim3(1), dim3(1), 0, b->stream, b->clk + 5, lambda, (int*)nullptr, 0);
    TRY(launch_check("k_set_value"));
    return batch_rhs(b, b->stream, b->clk + 5, x, dx);
}

pffrg_status pffrg_batch_flow(pffrg_batch* b, int n_lambda, const double* lambdas, double* x, int use_graph,
                              int* point_finite) {
    TRY(check_batch(b));
    if (!x || !lambdas) return fail(PFFRG_EINVAL, "null state or schedule");
    if (n_lambda < 2 || n_lambda > kMaxSchedule) return fail(PFFRG_EINVAL, "schedule needs 2 .. 65536 cutoffs");
    for (int i = 0; i < n_lambda; ++i)
        if (!(lambdas[i] > 0.0) || !std::isfinite(lambdas[i]))
            return fail(PFFRG_EINVAL, "cutoffs must be finite and > 0");
    HIP_TRY(hipStreamSynchronize(b->stream));
    HIP_TRY(hipMemcpy(b->sched, lambdas, sizeof(double) * n_lambda, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_set_value, dim3(1), dim3(1), 0, b->stream, (double*)nullptr, 0.0, b->step, 0);
    TRY(launch_check("k_set_value"));
    if (use_graph) {
        if (!b->exec || b->graph_x != x) TRY(capture_step(b, x));
        for (int i = 0; i + 1 < n_lambda; ++i) HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    } else {
        for (int i = 0; i + 1 < n_lambda; ++i) TRY(rk4_step(b, b->stream, x));
    }
    if (point_finite) TRY(finite_points(b, x, point_finite));
    return PFFRG_OK;
}

pffrg_status pffrg_batch_chi(pffrg_batch* b, double lambda, const double* x, double* chi) {
    TRY(check_batch(b));
    if (!x || !chi) return fail(PFFRG_EINVAL, "null pointer");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(PFFRG_EINVAL, "lambda must be finite and > 0");
    long co = 0;
    for (int p = 0; p < b->np; ++p) {
        const double* xp = x + b->pts[p].x_off;
        hipLaunchKernelGGL(k_chi_nodes, dim3(1), dim3(64), 0, b->stream, (const double*)b->w, b->nf, lambda, xp, b->cw,
                           b->cq, b->cg2, b->cn);
        TRY(launch_check("k_chi_nodes"));
        hipLaunchKernelGGL(k_chi_pairs, dim3(b->ns[p], kChiSlices), dim3(kChiThreads), 0, b->stream,
                           (const double*)b->w, b->nf, b->ns[p], (const int*)(b->swap + b->pts[p].pair_off), xp,
                           (const double*)b->cw, (const double*)b->cq, (const double*)b->cg2, (const int*)b->cn,
                           b->chi_part);
        TRY(launch_check("k_chi_pairs"));
        hipLaunchKernelGGL(k_chi_final, dim3(1), dim3(64), 0, b->stream, b->ns[p], (const double*)b->cq,
                           (const double*)b->cg2, (const int*)b->cn, (const double*)b->chi_part, chi + co);
        TRY(launch_check("k_chi_final"));
        co += 2 * b->ns[p];
    }
    return PFFRG_OK;
}

pffrg_status pffrg_batch_chi_k(pffrg_batch* b, int point, const double* chi, int nk, const double* kp, double* out) {
    TRY(check_batch(b));
    if (point < 0 || point >= b->np) return fail(PFFRG_EINVAL, "point out of range");
    if (nk < 0 || (nk > 0 && (!chi || !kp || !out))) return fail(PFFRG_EINVAL, "bad chi(k) arguments");
    if (nk == 0) return PFFRG_OK;
    hipLaunchKernelGGL(k_chi_k, dim3((nk + kChiKWaves - 1) / kChiKWaves), dim3(64 * kChiKWaves), 0, b->stream,
                       b->chi_cnt[point],
                       (const int*)(b->chi_pair + b->chi_off[point]), (const double*)(b->chi_dr + 3L * b->chi_off[point]),
                       1.0 / b->nb_chi[point], chi, 1, 0, 3.0, nk, kp, out);
    return launch_check("k_chi_k");
}

pffrg_status pffrg_batch_tune(pffrg_batch* b, double lambda, const double* x, int* per, int* order, int* split) {
    TRY(check_batch(b));
    if (!x) return fail(PFFRG_EINVAL, "null state");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(PFFRG_EINVAL, "lambda must be finite and > 0");
    const std::string key = tune_key(b->nf, b->ns, b->prec);
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) { b->cfg = it->second; have = true; }
    }
    if (!have) {
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        const bool prof = b->profiling;
        b->profiling = false;
        float best = 1e30f;
        LaunchCfg win = b->cfg;
        auto run = [&]() -> pffrg_status {
            for (int split = 0; split < 2; ++split)
            for (int order = 0; order < kOrders; ++order)
                for (int perv : {32, 64, 96, 128, 192, 256, 384, 512}) {
                    b->cfg = LaunchCfg{perv, order, split};
                    TRY(pffrg_batch_rhs(b, lambda, x, b->K));        // warm-up
                    HIP_TRY(hipEventRecord(e0, b->stream));
                    for (int r = 0; r < 3; ++r) TRY(pffrg_batch_rhs(b, lambda, x, b->K));
                    HIP_TRY(hipEventRecord(e1, b->stream));
                    HIP_TRY(hipEventSynchronize(e1));
                    float ms = 0.0f;
                    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best) { best = ms; win = b->cfg; }
                }
            return PFFRG_OK;
        };
        pffrg_status st = run();
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->profiling = prof;
        if (st != PFFRG_OK) return st;
        b->cfg = win;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[key] = win;
    }
    b->tuned = true;
    drop_graph(b);      // the step graph holds the old launch shape
    if (per) *per = b->cfg.per;
    if (order) *order = b->cfg.order;
    if (split) *split = b->cfg.split;
    return PFFRG_OK;
}

pffrg_status pffrg_batch_set_launch(pffrg_batch* b, int per, int order, int split) {
    TRY(check_batch(b));
    if (per < 1 || per > 4096 || order < 0 || order >= kOrders || split < 0 || split > 1)
        return fail(PFFRG_EINVAL, "bad launch shape");
    b->cfg = LaunchCfg{per, order, split};
    drop_graph(b);
    return PFFRG_OK;
}

pffrg_status pffrg_batch_set_profiling(pffrg_batch* b, int on) {
    TRY(check_batch(b));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->profiling = on != 0;
    b->ev_used = 0;
    drop_graph(b);      // events are recorded only by direct launches
    return PFFRG_OK;
}

pffrg_status pffrg_batch_profile_read(pffrg_batch* b, double* total_ms, int* count) {
    TRY(check_batch(b));
    if (!total_ms || !count) return fail(PFFRG_EINVAL, "null output");
    HIP_TRY(hipStreamSynchronize(b->stream));
    double tot = 0.0;
    for (int i = 0; i < b->ev_used; ++i) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, b->ev[2 * i], b->ev[2 * i + 1]));
        tot += ms;
    }
    *total_ms = tot;
    *count = b->ev_used;
    return PFFRG_OK;
}

}  // extern "C"
