// kernels_batch.h -- kernels that advance many flows at once (a scan over
// couplings and lattice ranges on one frequency mesh).
//
// Every point of a batch has its own symmetry-reduced lattice (pair count,
// exchange table, tabulated lattice sums) and its own flow state; the mesh,
// the Runge-Kutta schedule and the precision are shared.  The per-point
// arithmetic is the same as for one flow (the bodies of kernels_flow.h);
// what changes is how work reaches the GPU:
//   * sigma, node tables and packing are single launches over all points
//     (grid dimension y = point);
//   * the vertex right-hand side is one persistent launch: workgroups walk
//     a work list of tiles (point, four consecutive output triples, one per
//     wave) and each wave does all three channels of its triple, so the
//     derivative is written once.  The list is split into eight parts, one
//     per XCD; each point's tiles stay in one part so that the point's
//     vertex (a few MB) is read through one L2;
//   * the cutoffs of the Runge-Kutta stages come from device memory (a
//     clock record updated by a one-thread kernel), so one step can be
//     captured in a hipGraph and replayed.
#pragma once

#include "kernels_flow.h"

namespace pffrg {

// Where one point's tables, state and packed vertex sit in the batch-wide
// concatenated arrays.
struct BatchPoint {
    int ns, n_terms;
    int pair_off;      // into swap, mult, coupling (sum of ns of earlier points)
    int rpa_off_off;   // into rpa_off (sum of ns + 1)
    int term_off;      // into rpa_term
    long x_off;        // state offset in doubles
    long gv_off;       // packed vertex offset in elements
};

struct BatchArgs {
    FlowArgs base;           // mesh, nf, nq, su_a, su_c; table pointers of point 0
    const BatchPoint* pts;
    int n_points;
};

// Batch-wide limit of the pair count: one 2x4 register block per lane.
constexpr int kBatchMaxPairs = 20;

__device__ __forceinline__ FlowArgs point_args(const BatchArgs& B, int b) {
    const BatchPoint P = B.pts[b];
    FlowArgs A = B.base;
    A.ns = P.ns;
    A.n_terms = P.n_terms;
    A.swap = B.base.swap + P.pair_off;
    A.mult = B.base.mult + P.pair_off;
    A.rpa_off = B.base.rpa_off + P.rpa_off_off;
    A.rpa_term = B.base.rpa_term + P.term_off;
    const long tl = (long)b * 3 * A.nf;
    A.tab_n = B.base.tab_n + tl;
    A.tab_w = B.base.tab_w + tl * A.nq;
    A.tab_g = B.base.tab_g + tl * A.nq;
    return A;
}

__device__ __forceinline__ long point_vsz(const FlowArgs& A) {
    return (long)A.nf * (A.nf + 1) / 2 * A.nf * A.ns;
}

// Clock record: clk[0..3] = stage cutoffs of the current RK4 step
// (l0, l0 + h/2, l0 + h/2, l1), clk[4] = h = l1 - l0.  One thread.
static __global__ void k_batch_clock(const double* __restrict__ sched, const int* __restrict__ step,
                              double* __restrict__ clk) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int s = *step;
    const double l0 = sched[s], l1 = sched[s + 1];
    const double h = l1 - l0;
    const double lm = l0 + 0.5 * h;
    clk[0] = l0;
    clk[1] = lm;
    clk[2] = lm;
    clk[3] = l1;
    clk[4] = h;
}

static __global__ void k_batch_tick(int* __restrict__ step) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
}

static __global__ void k_set_value(double* __restrict__ p, double v, int* __restrict__ q, int iv) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    if (p) *p = v;
    if (q) *q = iv;
}

// grid (nf, points)
static __global__ void __launch_bounds__(kWave)
k_batch_sigma(BatchArgs B, const double* __restrict__ lamp, const double* __restrict__ x,
              double* __restrict__ dx) {
    const int b = blockIdx.y;
    FlowArgs A = point_args(B, b);
    const long off = B.pts[b].x_off;
    __shared__ MeshLds M;
    M.load(A, x + off, nullptr, threadIdx.x);
    A.w = M.w;
    sigma_body(A, *lamp, M.sig, x + off, point_vsz(A), dx + off, blockIdx.x, threadIdx.x);
}

// grid (3 nf, points); dx holds d sig of each point
static __global__ void __launch_bounds__(kWave)
k_batch_tables(BatchArgs B, const double* __restrict__ lamp, const double* __restrict__ x,
               const double* __restrict__ dx) {
    const int b = blockIdx.y;
    FlowArgs A = point_args(B, b);
    const long off = B.pts[b].x_off;
    __shared__ MeshLds M;
    M.load(A, x + off, dx + off, threadIdx.x);
    A.w = M.w;
    tables_body(A, *lamp, M.sig, M.dsig, blockIdx.x, threadIdx.x);
}

// grid (blocks, points): the packed vertex of every point
template <class R>
static __global__ void k_batch_pack(BatchArgs B, const double* __restrict__ x, V2<R>* __restrict__ gv) {
    const int b = blockIdx.y;
    const BatchPoint P = B.pts[b];
    const long n = (long)B.base.nf * (B.base.nf + 1) / 2 * B.base.nf * P.ns;
    const double* gs = x + P.x_off + B.base.nf;
    const double* gd = gs + n;
    V2<R>* out = gv + P.gv_off;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        V2<R> v;
        v.x = (R)gs[i];
        v.y = (R)gd[i];
        out[i] = v;
    }
}

// y = x + (am h) k and acc = (init ? x : acc) + (h / bdiv) k with h = clk[4]
// (the step's coefficients formed as in a single-flow step).
static __global__ void k_batch_rk_stage(long n, const double* __restrict__ x, const double* __restrict__ k, double am,
                                 double* __restrict__ y, double bdiv, double* __restrict__ acc, int init,
                                 const double* __restrict__ clk) {
    const double h = clk[4];
    const double a = am * h, bb = h / bdiv;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double ki = k[i], xi = x[i];
        if (y) y[i] = xi + a * ki;
        if (acc) acc[i] = (init ? xi : acc[i]) + bb * ki;
    }
}

// The persistent vertex launch.  items[i] = (point, first output triple of
// the tile); part x of the list (XCD x) is items[begin[x] .. begin[x+1]),
// walked by the per = gridDim.x / 8 workgroups of that XCD with stride per.
// LDS: shared tables at the front (shared_bytes, sized for the largest
// point), then one area of wave_bytes per wave.  PART selects the channels:
// kAll (s, u and t), kSU (s and u; writes dGamma) or kT (t; adds), so the
// right-hand side is one launch or two with smaller register needs.
constexpr int kAll = 0, kSU = 1, kT = 2;

// MAXNSP: the largest padded pair count the launch's points may have.  The
// split t launch runs the points of up to 16 pairs in an instance compiled
// for them alone (matrix-core lattice sum) and the larger ones in another;
// each fits four waves per SIMD, the one-launch kAll form three.
constexpr int kSmallNsp = 16;

template <class R, int PART, int MAXNSP = 20>
static __global__ void __launch_bounds__(kWave * kWavesPerBlock)
__attribute__((amdgpu_waves_per_eu(PART == kAll ? 3 : 4)))
k_batch_vertex(BatchArgs B, const V2<R>* __restrict__ gv, const int2* __restrict__ items,
               const int* __restrict__ begin, int shared_bytes, int wave_bytes, double* __restrict__ dx) {
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int per = gridDim.x / 8;
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    unsigned char* base = lds_raw + shared_bytes + wid * wave_bytes;
    const int i1 = begin[xcd + 1];
    int cur = -1;
    for (int i = begin[xcd] + slot; i < i1; i += per) {
        // only the point index is carried from tile to tile; the point's
        // arguments are re-read (scalar loads) to keep register pressure low
        const int2 item = items[i];
        FlowArgs A = point_args(B, item.x);
        if (item.x != cur) {                 // uniform over the workgroup
            __syncthreads();
            fill_shared<false>(A, lds_raw, PART != kSU);
            cur = item.x;
        }
        const Shared sh = shared_ptrs(A, lds_raw);
        A.w = sh.w;
        const long x_off = B.pts[item.x].x_off, gv_off = B.pts[item.x].gv_off;
        const int nf = A.nf, ns = A.ns;
        const int n_triples = nf * (nf + 1) / 2 * nf;
        const int o = __builtin_amdgcn_readfirstlane(item.y + wid);    // wave-uniform
        if (o < n_triples) {
            const int su = o / nf, it = o % nf;
            const Triple T = make_triple(A.w, nf, A.su_a[su], it, A.su_c[su]);
            const __amdgpu_buffer_rsrc_t rv = vertex_rsrc<R>(gv + gv_off, (long)n_triples * ns);
            const WaveLds<R> L{ns, kSub};
            double* red = reinterpret_cast<double*>(base + L.mat());
            const long vsz = (long)n_triples * ns;
            double* out = dx + x_off + nf;
            const int G = kWave / ns;
            const bool act = lane / ns < G;
            // s + u are finished (written) before t is added, in every
            // launch shape, so all shapes give the same bits
            if (PART != kT) {
                SuPart ps = su_body<0, R>(A, sh, reinterpret_cast<PlanT<R>*>(base), T, rv, lane);
                const SuPart pu = su_body<2, R>(A, sh, reinterpret_cast<PlanT<R>*>(base), T, rv, lane);
                for (int h = 0; h < 2; ++h) {
                    ps.s[h] += pu.s[h];
                    ps.d[h] += pu.d[h];
                }
                finish_su<R>(red, lane, ns, ps, out + T.out * ns, out + vsz + T.out * ns, false);
                wave_lds_sync();
            }
            if (PART != kSU) {
                LanePart pt{0.0, 0.0};
                // the large-pair t launch holds the 20-pair body alone, which
                // keeps it within the registers of four waves per SIMD
                if constexpr (PART == kT && MAXNSP > kSmallNsp) pt = t_body<20, R>(A, sh, base, T, rv, lane);
                else switch ((ns + 3) / 4) {
                    case 1: pt = t_body<4, R>(A, sh, base, T, rv, lane); break;
                    case 2: pt = t_body<8, R>(A, sh, base, T, rv, lane); break;
                    case 3: pt = t_body<12, R>(A, sh, base, T, rv, lane); break;
                    case 4: pt = t_body<16, R>(A, sh, base, T, rv, lane); break;
                    default:
                        if constexpr (MAXNSP > kSmallNsp) pt = t_body<20, R>(A, sh, base, T, rv, lane);
                        break;
                }
                finish_pairs(red, lane, ns, G, act, pt.s, pt.d, 0.0, 0.0, out + T.out * ns,
                             out + vsz + T.out * ns, true);
            }
        }
    }
}

}  // namespace pffrg
