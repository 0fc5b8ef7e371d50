// kernels_flow.h -- HIP kernels of the SU(2) pf-FRG right-hand side (gfx950).
//
// One right-hand side (arXiv:2109.13317, Sec. 3) is four launches:
//   k_sigma_rhs     d sig/d Lambda on the mesh (Eq. 23): the single-scale
//                   propagator pins the internal frequency to +-Lambda; one
//                   wave per mesh frequency, lanes over pairs;
//   k_tables_pack   per channel X in {s,t,u} and transfer frequency index nu,
//                   the evaluation points w_k of the channel's frequency
//                   integral and their weights W_k (delta points of S and
//                   trapezoid nodes of the Katanin term, Eq. 13), so that the
//                   channel integral is sum_k W_k F_X(w_k), one wave per list;
//                   the remaining workgroups interleave the two vertex
//                   strains as (Gs, Gd) pairs, so that one interpolation
//                   corner is one 16-byte load;
//   k_vertex_stu    the three channel sums of every output triple (s,t,u) for
//                   every pair, one wave per triple; its workgroups take the
//                   s, u and t roles in turn, so every CU runs all three: the
//                   t role (the particle-hole lattice sum in GEMM form,
//                   M = sum_k W_k a_k b_k^T, register-blocked 2x4 per lane,
//                   contracted with the tabulated (ka, kb, count) terms) is
//                   bound by the vector ALU and load latency, the s and u
//                   roles by the rate of gather instructions, and mixed on
//                   one CU they overlap;
//   k_sum_channels  dGamma = (s part + u part) + t part.
// The same channel bodies run as three launches (k_vertex_su<0> writes,
// k_vertex_su<2> and k_vertex_t<NSP> add, in that order: the same sums
// bitwise) where each channel is timed on its own.
#pragma once

#include "device_common.h"

namespace pffrg {

struct FlowArgs {
    const double* w;        // mesh [nf]
    int nf, ns, nq;         // mesh size, pairs, node-table stride
    const int* swap;        // [ns]
    const int* mult;        // [ns]
    const int* rpa_off;     // [ns+1]
    const int* rpa_ka;
    const int* rpa_kb;
    const int* rpa_cnt;
    const int* rpa_term;    // packed terms (ka*ns + kb) | (count << 16), rpa_off order
    int n_terms;
    const int* su_a;        // [nf(nf+1)/2] s-index of each (s,u) wedge entry
    const int* su_c;        //              u-index
    int* tab_n;             // [3*nf] node counts
    double* tab_w;          // [3*nf*nq] node frequencies
    double* tab_g;          // [3*nf*nq] node weights
    const unsigned char* lut;   // [kLutMax] mesh look-up table (build_mesh_lut)
    int lut_shift, lut_kmin;
    const int2* run;        // [kWave] term runs (term_runs), or null
    const int* run_off;     // [ns+1]
};

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Order LDS traffic between lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The packed vertex: the two strains of one element side by side, in the
// precision R the vertex kernels work in (double2, or float2 in FP32 mode).
template <class R> struct Packed;
template <> struct Packed<double> { using V2 = double2; using V4 = double4; };
template <> struct Packed<float> { using V2 = float2; using V4 = float4; };
template <class R> using V2 = typename Packed<R>::V2;
template <class R> using V4 = typename Packed<R>::V4;
template <class R> constexpr int kElemBytes = 2 * (int)sizeof(R);

__device__ __forceinline__ double fmr(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmr(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Buffer resource of the packed vertex: loads take a 32-bit byte offset;
// reads past the end return 0 (they never happen: every plan offset lies in
// the state).  Base and size are the same for the whole wave (one context,
// or one batch point per wave) and are made wave-uniform explicitly: a
// descriptor the compiler cannot prove uniform (a batch point's offset read
// from memory) costs a readfirstlane loop around every load.
template <class R>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vertex_rsrc(const V2<R>* gv, long n) {
    const unsigned long long a = reinterpret_cast<unsigned long long>(gv);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)a);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
    void* base = reinterpret_cast<void*>(((unsigned long long)hi << 32) | lo);
    const int bytes = __builtin_amdgcn_readfirstlane((int)(n * kElemBytes<R>));
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, bytes, 0x00020000);
}

__device__ __forceinline__ double2 load_corner(__amdgpu_buffer_rsrc_t r, unsigned byte_off, double) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0));
}
__device__ __forceinline__ float2 load_corner(__amdgpu_buffer_rsrc_t r, unsigned byte_off, float) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0));
}

// Interpolation of both strains of one pair from the packed vertex; plan
// offsets are byte offsets, pp = element bytes * (p, swap[p]).
template <class R>
__device__ __forceinline__ void eval_packed2(const PlanT<R>& P, __amdgpu_buffer_rsrc_t r, int2 pp,
                                             R& vs, R& vd) {
    const unsigned q = P.swp ? pp.y : pp.x;
    R a = 0, b = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const V2<R> g = load_corner(r, (unsigned)P.off[i] + q, R());
        a = fmr(P.ws[i], g.x, a);
        b = fmr(P.wd[i], g.y, b);
    }
    vs = a;
    vd = b;
}

// Two interpolations (plans Pa and Pb, pair offsets pp) with all eight corner
// loads issued before any arithmetic, so they are in flight together.
template <class R>
__device__ __forceinline__ void eval_packed_ab(const PlanT<R>& Pa, const PlanT<R>& Pb, __amdgpu_buffer_rsrc_t r,
                                               int2 pp, R& as, R& ad, R& bs, R& bd) {
    const unsigned qa = Pa.swp ? pp.y : pp.x, qb = Pb.swp ? pp.y : pp.x;
    V2<R> ga[4], gb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ga[i] = load_corner(r, (unsigned)Pa.off[i] + qa, R());
#pragma unroll
    for (int i = 0; i < 4; ++i) gb[i] = load_corner(r, (unsigned)Pb.off[i] + qb, R());
    R a0 = 0, a1 = 0, b0 = 0, b1 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        a0 = fmr(Pa.ws[i], ga[i].x, a0);
        a1 = fmr(Pa.wd[i], ga[i].y, a1);
        b0 = fmr(Pb.ws[i], gb[i].x, b0);
        b1 = fmr(Pb.wd[i], gb[i].y, b1);
    }
    as = a0; ad = a1; bs = b0; bd = b1;
}

// The same two evaluations through fraction plans (FP64): the corner weights
// are formed here, after the loads are issued.
__device__ __forceinline__ void frac_apply(const FracPlan& P, const double2 (&g)[4], double& vs, double& vd) {
    const double u0 = 1.0 - P.t0, u1 = 1.0 - P.t1;
    const double wg[4] = {u0 * u1, u0 * P.t1, P.t0 * u1, P.t0 * P.t1};
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        a = fmr(wg[i], g[i].x, a);
        b = fmr((P.flags >> i) & 1 ? -wg[i] : wg[i], g[i].y, b);
    }
    vs = a;
    vd = b;
}
__device__ __forceinline__ void eval_packed2(const FracPlan& P, __amdgpu_buffer_rsrc_t r, int2 pp, double& vs,
                                             double& vd) {
    const unsigned q = P.flags & 16 ? pp.y : pp.x;
    double2 g[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) g[i] = load_corner(r, (unsigned)P.off[i] + q, double());
    frac_apply(P, g, vs, vd);
}
__device__ __forceinline__ void eval_packed_ab(const FracPlan& Pa, const FracPlan& Pb, __amdgpu_buffer_rsrc_t r,
                                               int2 pp, double& as, double& ad, double& bs, double& bd) {
    const unsigned qa = Pa.flags & 16 ? pp.y : pp.x, qb = Pb.flags & 16 ? pp.y : pp.x;
    double2 ga[4], gb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ga[i] = load_corner(r, (unsigned)Pa.off[i] + qa, double());
#pragma unroll
    for (int i = 0; i < 4; ++i) gb[i] = load_corner(r, (unsigned)Pb.off[i] + qb, double());
    frac_apply(Pa, ga, as, ad);
    frac_apply(Pb, gb, bs, bd);
}

// A plan whose offsets are turned into byte offsets of the packed vertex.
template <class R>
__device__ __forceinline__ void to_bytes(PlanT<R>& P) {
#pragma unroll
    for (int i = 0; i < 4; ++i) P.off[i] *= kElemBytes<R>;
}
__device__ __forceinline__ void to_bytes(FracPlan& P) {
#pragma unroll
    for (int i = 0; i < 4; ++i) P.off[i] *= kElemBytes<double>;
}

// The t channel's plans: in FP64 fraction plans (under half the LDS bytes
// read per evaluation, and fewer live registers: the kernels up to 16 pairs
// hold five waves per SIMD without spilling); in FP32 the float weights of
// PlanT<float> are already compact.
template <class R> struct TPlanOf { using type = PlanT<R>; };
template <> struct TPlanOf<double> { using type = FracPlan; };
template <class R> using TPlan = typename TPlanOf<R>::type;

// Running sum of per-chunk partial sums.  In FP32 the rounding error of each
// addition is carried along (Kahan's compensated summation) and the value is
// s - c evaluated in FP64; in FP64 it is a plain sum.
template <class R>
struct CompSum {
    R s = 0, c = 0;
    __device__ __forceinline__ void add(R x) {
        if constexpr (sizeof(R) == 4) {
            const R y = x - c;
            const R t = s + y;
            c = (t - s) - y;
            s = t;
        } else {
            s += x;
        }
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// ------------------------------------------------------------ self-energy -

// d sig/d Lambda (w_n) = (1/2pi) sum_{x=+-Lambda} F(w_n, x) / (x - sig(x)),
// F = 2 sum_r mult_r Gd_r(w+x, 0, w-x) - 3 Gs_0(w+x, x-w, 0) - Gd_0(w+x, x-w, 0).
// sig: the self-energy values (may be an LDS copy of x[0 .. nf)).
__device__ __forceinline__ void sigma_body(const FlowArgs& A, double lam, const double* __restrict__ sig,
                                           const double* __restrict__ x, long nv, double* __restrict__ dsig,
                                           int n, int lane) {
    const double wn = A.w[n];
    const double* gs = x + A.nf;
    const double* gd = gs + nv;
    // lanes 0..31 take x = +Lambda, lanes 32..63 x = -Lambda; lane r of a
    // half reads pair r (at most 32 pairs), its lane 0 also the on-site terms
    const int half = lane >> 5, r = lane & 31;
    const double xx = half == 0 ? lam : -lam;
    Plan P;
    make_plan(A.w, A.nf, A.ns, wn + xx, 0.0, wn - xx, 1, 0, P);
    double f = 0.0;
    if (r < A.ns) {
        double vs, vd;
        eval_plan(P, gs, gd, A.swap, r, vs, vd);
        f = 2.0 * (double)A.mult[r] * vd;
    }
    if (r == 0) {
        Plan Q;
        make_plan(A.w, A.nf, A.ns, wn + xx, xx - wn, 0.0, 2, 0, Q);
        double os, od;
        eval_plan(Q, gs, gd, A.swap, 0, os, od);
        f -= 3.0 * os + od;
    }
    for (int o = 16; o > 0; o >>= 1) f += __shfl_xor(f, o, kWave);
    const double term = f / (xx - odd_interp(A.w, A.nf, sig, xx));
    const double other = __shfl(term, 32, kWave);
    if (lane == 0) dsig[n] = (term + other) * kInvTwoPi;
}

// Mesh, self-energy and (optionally) its derivative copied to LDS by one
// wave: the binary searches of the look-ups then never touch memory.
struct MeshLds {
    double w[128], sig[128], dsig[128];
    __device__ __forceinline__ void load(const FlowArgs& A, const double* sig_g, const double* dsig_g, int lane) {
        for (int i = lane; i < A.nf; i += kWave) {
            w[i] = A.w[i];
            sig[i] = sig_g[i];
            if (dsig_g) dsig[i] = dsig_g[i];
        }
        __syncthreads();
    }
};

static __global__ void __launch_bounds__(kWave)
k_sigma_rhs(FlowArgs A, double lam, const double* __restrict__ x, long nv, double* __restrict__ dsig) {
    __shared__ MeshLds M;
    M.load(A, x, nullptr, threadIdx.x);
    A.w = M.w;
    sigma_body(A, lam, M.sig, x, nv, dsig, blockIdx.x, threadIdx.x);
}

template <class R>
static __global__ void k_pack(long n, const double* __restrict__ gs, const double* __restrict__ gd,
                       V2<R>* __restrict__ gv) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        V2<R> v;
        v.x = (R)gs[i];
        v.y = (R)gd[i];
        gv[i] = v;
    }
}

// ------------------------------------------------------------ node tables -

// Channel partner frequency: s: nu - w, t: w - nu, u: nu + w.
__device__ __forceinline__ double partner(int ch, double nu, double w) {
    return ch == 0 ? nu - w : (ch == 1 ? w - nu : nu + w);
}

// Step function of a propagator evaluated at a delta point: 1 outside,
// 1/2 exactly on the edge |y| == Lambda.
__device__ __forceinline__ double theta_half(double y, double lam) {
    const double a = fabs(y);
    return a > lam ? 1.0 : (a == lam ? 0.5 : 0.0);
}

// The full mesh -w[nf-1] .. -w[0], w[0] .. w[nf-1], ascending.
__device__ __forceinline__ double full_mesh(const double* __restrict__ w, int nf, int i) {
    return i < nf ? -w[nf - 1 - i] : w[i - nf];
}

// Number of full-mesh points that are <= x (le) or < x (!le).
__device__ __forceinline__ int full_mesh_count(const double* __restrict__ w, int nf, double x, bool le) {
    int lo = 0, hi = 2 * nf;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const double v = full_mesh(w, nf, mid);
        if (le ? v <= x : v < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One wave per (channel, nu).  Node list: the delta points first, then for
// every piece of D = [-wmax, wmax] \ (-lam, lam) \ (c - lam, c + lam) (c = zero
// of the partner) its ends and the mesh points strictly inside, with
// trapezoid weight times the Katanin bubble.  The four delta candidates and
// the four pieces are worked out on lanes 0..3 at once; the nodes of all
// pieces are then spread over the wave.  The walk is shared by the table
// builder and its vector-Jacobian product: V receives
//   delta(n, node, x, y, theta)  node n = w at a delta point x = +-Lambda,
//       weight -theta / ((x - sig(x)) (y - sig(y))) / (2 pi) with y the
//       frequency of the other propagator (called by one lane per node);
//   kat(n, w, partner(w), trapezoid weight)  one Katanin node (per lane);
//   done(n, lane)  the list length.
template <class V>
__device__ __forceinline__ void walk_nodes(const FlowArgs& A, double lam, int id, int lane, V& vis) {
    const int nf = A.nf;
    const int ch = id / nf, iv = id % nf;
    const double nu = A.w[iv];

    // delta parts (lane 2 sx + k, x = +Lambda then -Lambda): the S in
    // Skat(partner(w)) puts w at partner^-1(x) (k = 0); the S in Skat(w) puts
    // w at x (k = 1)
    int nd;
    {
        double node = 0.0, xx = 0.0, y = 0.0, th = 0.0;
        if (lane < 4) {
            xx = (lane >> 1) == 0 ? lam : -lam;
            if ((lane & 1) == 0) {
                node = ch == 0 ? nu - xx : (ch == 1 ? xx + nu : xx - nu);
                y = node;
            } else {
                node = xx;
                y = partner(ch, nu, xx);
            }
            th = theta_half(y, lam);
        }
        const bool on = lane < 4 && th != 0.0;
        const unsigned long long mask = __ballot(on);
        if (on) vis.delta(__popcll(mask & ((1ull << lane) - 1ull)), node, xx, y, th);
        nd = __popcll(mask);
    }

    // pieces (lane 2 ip + q): [lo, hi], the full-mesh points up to lo and
    // the node count m (the two ends and the mesh points strictly inside)
    const double c = ch == 0 ? nu : (ch == 1 ? nu : -nu);
    const double wmax = A.w[nf - 1];
    const double e0 = c - lam, e1 = c + lam;
    double lo = 0.0, hi = 0.0;
    int below = 0, m = 0;
    if (lane < 4) {
        const int ip = lane >> 1, q = lane & 1;
        const double a = ip == 0 ? -wmax : lam, b = ip == 0 ? -lam : wmax;
        if (a < b) {
            lo = q == 0 ? a : (a > e1 ? a : e1);
            hi = q == 0 ? (b < e0 ? b : e0) : b;
            if (lo < hi) {
                below = full_mesh_count(A.w, nf, lo, true);
                m = full_mesh_count(A.w, nf, hi, false) - below + 2;
            }
        }
    }
    double plo[4], phi[4];
    int pbelow[4], pm[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        plo[k] = __shfl(lo, k, kWave);
        phi[k] = __shfl(hi, k, kWave);
        pbelow[k] = __shfl(below, k, kWave);
        pm[k] = __shfl(m, k, kWave);
    }
    const int total = pm[0] + pm[1] + pm[2] + pm[3];
    for (int j = lane; j < total; j += kWave) {
        int k = 0, base = 0;
#pragma unroll
        for (int kk = 1; kk < 4; ++kk)
            if (j >= base + pm[k]) { base += pm[k]; k = kk; }
        double l = plo[0], h = phi[0];
        int bl = pbelow[0], mm = pm[0];
#pragma unroll
        for (int kk = 1; kk < 4; ++kk)
            if (k == kk) { l = plo[kk]; h = phi[kk]; bl = pbelow[kk]; mm = pm[kk]; }
        const int jj = j - base;
        auto node = [&](int q) { return q == 0 ? l : (q == mm - 1 ? h : full_mesh(A.w, nf, bl + q - 1)); };
        const double cur = node(jj);
        const double wl = jj > 0 ? 0.5 * (cur - node(jj - 1)) : 0.0;
        const double wr = jj + 1 < mm ? 0.5 * (node(jj + 1) - cur) : 0.0;
        vis.kat(nd + j, cur, partner(ch, nu, cur), wl + wr);
    }
    vis.done(nd + total, lane);
}

// Writes the node list (frequencies tw, weights tg, length tn).
struct TableWriter {
    const double* w;
    int nf;
    const double* sig;
    const double* dsig;
    double* tw;
    double* tg;
    int* tn;
    __device__ __forceinline__ void delta(int n, double node, double xx, double y, double th) {
        const double st = 1.0 / (xx - odd_interp(w, nf, sig, xx));
        const double g = th / (y - odd_interp(w, nf, sig, y));
        tw[n] = node;
        tg[n] = -st * g * kInvTwoPi;
    }
    __device__ __forceinline__ void kat(int n, double cur, double pp, double wt) {
        const double gw = 1.0 / (cur - odd_interp(w, nf, sig, cur));
        const double gp = 1.0 / (pp - odd_interp(w, nf, sig, pp));
        const double k = gw * gp * gp * odd_interp(w, nf, dsig, pp) + gp * gw * gw * odd_interp(w, nf, dsig, cur);
        tw[n] = cur;
        tg[n] = wt * k * kInvTwoPi;
    }
    __device__ __forceinline__ void done(int n, int lane) {
        if (lane == 0) *tn = n;
    }
};

__device__ __forceinline__ void tables_body(const FlowArgs& A, double lam, const double* __restrict__ x,
                                            const double* __restrict__ dsig, int id, int lane) {
    TableWriter wr{A.w, A.nf, x, dsig, A.tab_w + (long)id * A.nq, A.tab_g + (long)id * A.nq, A.tab_n + id};
    walk_nodes(A, lam, id, lane, wr);
}

static __global__ void __launch_bounds__(kWave)
k_node_tables(FlowArgs A, double lam, const double* __restrict__ x, const double* __restrict__ dsig) {
    __shared__ MeshLds M;
    M.load(A, x, dsig, threadIdx.x);
    A.w = M.w;
    tables_body(A, lam, M.sig, M.dsig, blockIdx.x, threadIdx.x);
}

// The node tables and the packed vertex in one launch (both only read the
// state): the first 3 nf workgroups build one node list each, the others
// pack kPackPerLane elements per lane, so the bandwidth-bound packing runs
// beside the latency-bound tables instead of after them.
constexpr int kPackPerLane = 4;

template <class R>
static __global__ void __launch_bounds__(kWave)
k_tables_pack(FlowArgs A, double lam, const double* __restrict__ x, const double* __restrict__ dsig, long nv,
              V2<R>* __restrict__ gv) {
    const int n_lists = 3 * A.nf;
    if ((int)blockIdx.x < n_lists) {
        __shared__ MeshLds M;
        M.load(A, x, dsig, threadIdx.x);
        A.w = M.w;
        tables_body(A, lam, M.sig, M.dsig, blockIdx.x, threadIdx.x);
        return;
    }
    const double* gs = x + A.nf;
    const double* gd = gs + nv;
    const long base = (long)(blockIdx.x - n_lists) * (kWave * kPackPerLane) + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kPackPerLane; ++j) {
        const long i = base + (long)j * kWave;
        if (i < nv) {
            V2<R> v;
            v.x = (R)gs[i];
            v.y = (R)gd[i];
            gv[i] = v;
        }
    }
}

// ------------------------------------------------------------- vertex RHS -
//
// The vertex right-hand side is three launches, one per channel, each with
// its own order of the output triples so that the workgroups resident on one
// XCD (and its L2) share the frequency slice their channel interpolates in:
// s channel by s, u channel by u, t channel by t.  The s launch writes dGamma,
// the u and t launches add to it.

constexpr int kWavesPerBlock = 4;
constexpr int kPlanChunk = 32;   // s/u channels: nodes whose plans are built at once (two vectors each)
constexpr int kTChunk = 16;      // t channel: nodes whose four plans (two vectors, two on-site) are built at once
constexpr int kSub = 8;          // nodes per lattice-sum sub-chunk
constexpr int kMaxPairs = 32;    // 2 register blocks of 2x4 per lane cover 32 x 32
constexpr int kMaxFreq = 128;    // mesh copy in LDS

// Workgroup-shared tables in LDS: mesh, reciprocal spacings, the mesh look-up
// table, pair exchange, and (t channel) the packed tabulated lattice-sum
// terms with their offsets and their split into runs (term_runs).
struct SharedLds {
    int nf, ns, n_terms;
    __host__ __device__ size_t mesh() const { return 0; }
    __host__ __device__ size_t ih() const { return (size_t)nf * sizeof(double); }
    __host__ __device__ size_t lut() const { return (size_t)2 * nf * sizeof(double); }
    __host__ __device__ size_t swap() const { return lut() + kLutMax; }
    __host__ __device__ size_t off() const { return swap() + (size_t)ns * sizeof(int); }
    __host__ __device__ size_t terms() const { return off() + (size_t)(ns + 1) * sizeof(int); }
    __host__ __device__ size_t runs() const { return (terms() + (size_t)n_terms * sizeof(int) + 7) & ~(size_t)7; }
    __host__ __device__ size_t run_off() const { return runs() + (size_t)kWave * sizeof(int2); }
    __host__ __device__ size_t bytes(bool with_terms) const {
        const size_t b = with_terms ? run_off() + (size_t)(ns + 1) * sizeof(int) : terms();
        return (b + 31) & ~(size_t)31;
    }
};

struct Shared {
    const double* w;
    MeshLut lut;    // reciprocal spacings and look-up table in LDS
    const int* swap;
    const int* off;
    const int* terms;
    const int2* run;     // [kWave] term runs [x, y) (term_runs; filled on request, see fill_shared)
    const int* run_off;  // [ns+1] runs of pair p: run_off[p] .. run_off[p+1]-1
};

// Pointers to the shared tables in LDS (no memory traffic).
__device__ __forceinline__ Shared shared_ptrs(const FlowArgs& A, unsigned char* lds) {
    const SharedLds S{A.nf, A.ns, A.n_terms};
    return Shared{reinterpret_cast<double*>(lds + S.mesh()),
                  MeshLut{reinterpret_cast<double*>(lds + S.ih()), lds + S.lut(), A.lut_shift, A.lut_kmin},
                  reinterpret_cast<int*>(lds + S.swap()), reinterpret_cast<int*>(lds + S.off()),
                  reinterpret_cast<int*>(lds + S.terms()), reinterpret_cast<int2*>(lds + S.runs()),
                  reinterpret_cast<int*>(lds + S.run_off())};
}

// The tabulated terms of the lattice sum split into at most 64 runs of
// near-equal length, each within one output pair (host side, once per
// context): pair p gets k_p runs, one more at a time to the pair whose runs
// are longest.  Run r covers terms [run[2r], run[2r+1]), the runs of pair p
// are run_off[p] .. run_off[p+1]-1, and runs past the last are empty.  Lane
// r of a contraction takes run r, so no lane waits on the pair with the
// most terms.  Returns the number of runs (at most kWave; ns <= kWave).
inline int term_runs(int ns, const int* off, int* run, int* run_off) {
    int k[kWave];
    int total = 0;
    for (int p = 0; p < ns; ++p) {
        k[p] = off[p + 1] > off[p] ? 1 : 0;
        total += k[p];
    }
    while (total < kWave) {
        int best = -1, len = 0;
        for (int p = 0; p < ns; ++p) {
            const int n = off[p + 1] - off[p];
            if (k[p] == 0 || k[p] >= n) continue;
            const int l = (n + k[p] - 1) / k[p];
            if (l > len) { len = l; best = p; }
        }
        if (best < 0 || len <= 1) break;
        ++k[best];
        ++total;
    }
    int s = 0;
    for (int p = 0; p < ns; ++p) {
        run_off[p] = s;
        const int n = off[p + 1] - off[p];
        for (int i = 0; i < k[p]; ++i, ++s) {
            run[2 * s] = off[p] + (int)((long)n * i / k[p]);
            run[2 * s + 1] = off[p] + (int)((long)n * (i + 1) / k[p]);
        }
    }
    run_off[ns] = s;
    for (int r = s; r < kWave; ++r) run[2 * r] = run[2 * r + 1] = 0;
    return s;
}

// Fill the shared tables (workgroup-wide; before any wave leaves); with_runs
// also copies the term runs (the t channel beyond 20 pairs).  Each thread
// issues every global load of the first pass (one index of each table and up
// to kFillTerms terms) before its first LDS write, so the workgroup waits on
// about one load latency instead of one per table and pass; what the first
// pass leaves (long meshes, many terms, small workgroups) is copied after it
// in strided loops.  kFirst = false (a fill inside a persistent loop, where
// the first pass's registers would spill) copies each table in its own loop
// and no runs.
constexpr int kFillTerms = 16;
template <bool kFirst = true>
__device__ __forceinline__ void fill_shared(const FlowArgs& A, unsigned char* lds, bool with_terms,
                                            bool with_runs = false) {
    const Shared sh = shared_ptrs(A, lds);
    double* w = const_cast<double*>(sh.w);
    double* ih = const_cast<double*>(sh.lut.ih);
    unsigned* lut = reinterpret_cast<unsigned*>(const_cast<unsigned char*>(sh.lut.lut));
    int* sw = const_cast<int*>(sh.swap);
    int* off = const_cast<int*>(sh.off);
    int* terms = const_cast<int*>(sh.terms);
    if constexpr (!kFirst) {
        for (int i = threadIdx.x; i < A.nf; i += blockDim.x) {
            w[i] = A.w[i];
            ih[i] = i + 1 < A.nf ? 1.0 / (A.w[i + 1] - A.w[i]) : 0.0;
        }
        for (int i = threadIdx.x; i < kLutMax / 4; i += blockDim.x) lut[i] = reinterpret_cast<const unsigned*>(A.lut)[i];
        for (int i = threadIdx.x; i < A.ns; i += blockDim.x) sw[i] = A.swap[i];
        if (with_terms) {
            for (int i = threadIdx.x; i <= A.ns; i += blockDim.x) off[i] = A.rpa_off[i];
            for (int i = threadIdx.x; i < A.n_terms; i += blockDim.x) terms[i] = A.rpa_term[i];
        }
        __syncthreads();
        return;
    }
    const unsigned* lsrc = reinterpret_cast<const unsigned*>(A.lut);
    int2* run = const_cast<int2*>(sh.run);
    int* roff = const_cast<int*>(sh.run_off);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nf = A.nf, ns = A.ns, nterm = A.n_terms;
    // first pass: loads
    double w0 = 0.0, w1 = 0.0;
    unsigned lv = 0u;
    int sv = 0, ov = 0, rov = 0;
    int2 rv = make_int2(0, 0);
    int tv[kFillTerms];
    if (tid < nf) {
        w0 = A.w[tid];
        if (tid + 1 < nf) w1 = A.w[tid + 1];
    }
    if (tid < kLutMax / 4) lv = lsrc[tid];
    if (tid < ns) sv = A.swap[tid];
    if (with_terms) {
        if (tid <= ns) ov = A.rpa_off[tid];
#pragma unroll
        for (int k = 0; k < kFillTerms; ++k) {
            const int i = tid + k * nt;
            tv[k] = i < nterm ? A.rpa_term[i] : 0;
        }
        if (with_runs) {
            if (tid < kWave) rv = A.run[tid];
            if (tid <= ns) rov = A.run_off[tid];
        }
    }
    // first pass: stores
    if (tid < nf) {
        w[tid] = w0;
        ih[tid] = tid + 1 < nf ? 1.0 / (w1 - w0) : 0.0;
    }
    if (tid < kLutMax / 4) lut[tid] = lv;
    if (tid < ns) sw[tid] = sv;
    if (with_terms) {
        if (tid <= ns) off[tid] = ov;
#pragma unroll
        for (int k = 0; k < kFillTerms; ++k) {
            const int i = tid + k * nt;
            if (i < nterm) terms[i] = tv[k];
        }
        if (with_runs) {
            if (tid < kWave) run[tid] = rv;
            if (tid <= ns) roff[tid] = rov;
        }
    }
    // the rest
    for (int i = tid + nt; i < nf; i += nt) {
        w[i] = A.w[i];
        ih[i] = i + 1 < nf ? 1.0 / (A.w[i + 1] - A.w[i]) : 0.0;
    }
    for (int i = tid + nt; i < kLutMax / 4; i += nt) lut[i] = lsrc[i];
    for (int i = tid + nt; i < ns; i += nt) sw[i] = A.swap[i];
    if (with_terms) {
        for (int i = tid + nt; i <= ns; i += nt) off[i] = A.rpa_off[i];
        for (int i = tid + kFillTerms * nt; i < nterm; i += nt) terms[i] = A.rpa_term[i];
        if (with_runs) {
            for (int i = tid + nt; i < kWave; i += nt) run[i] = A.run[i];
            for (int i = tid + nt; i <= ns; i += nt) roff[i] = A.run_off[i];
        }
    }
    __syncthreads();
}

__device__ __forceinline__ Shared load_shared(const FlowArgs& A, unsigned char* lds, bool with_terms,
                                              bool with_runs = false) {
    fill_shared(A, lds, with_terms, with_runs);
    return shared_ptrs(A, lds);
}

// Pairs per lane in the s/u channels: FP64 one (a 16-byte corner load per
// pair); FP32 two adjacent pairs, whose packed elements one 16-byte load
// fetches together, so a node takes half the load instructions.
template <class R> constexpr int kSuPairs = sizeof(R) == 4 ? 2 : 1;

// Per-wave LDS of the t-channel kernel, in bytes (R: the vertex precision).
// The lattice-sum matrix at the end reuses it.  The s/u kernel uses
// plans() + red().
template <class R>
struct WaveLds {
    int ns;
    int sub = kSub;   // nodes per lattice-sum sub-chunk
    __host__ __device__ int nsp() const { return (ns + 3) & ~3; }
    __host__ __device__ size_t plans() const { return (size_t)2 * kTChunk * sizeof(TPlan<R>); }
    __host__ __device__ size_t onsite() const { return (((size_t)5 * kTChunk * sizeof(R)) + 15) & ~(size_t)15; }
    __host__ __device__ size_t su_plans() const { return (size_t)2 * kPlanChunk * sizeof(PlanT<R>); }
    __host__ __device__ size_t su_w() const { return (size_t)kPlanChunk * sizeof(double); }
    __host__ __device__ size_t vbuf() const { return (size_t)4 * sub * nsp() * sizeof(R); }
    __host__ __device__ size_t red() const { return (size_t)2 * kSuPairs<R> * kWave * sizeof(double); }
    __host__ __device__ size_t mat() const { return (((size_t)ns * ns * sizeof(double)) + 31) & ~(size_t)31; }
    __host__ __device__ size_t work() const { return plans() + onsite() + vbuf(); }
    __host__ __device__ size_t bytes() const {
        size_t m = mat() + red();
        size_t b = work() > m ? work() : m;
        return (b + 31) & ~(size_t)31;
    }
    __host__ __device__ size_t su_bytes() const { return ((su_plans() + su_w() + 31) & ~(size_t)31) + red(); }
    // an area that serves both bodies (one wave doing s, u and t in turn)
    __host__ __device__ size_t all_bytes() const { return bytes() > su_bytes() ? bytes() : su_bytes(); }
};

// Position in the channel's order of the triple handled by this wave, or -1.
// Consecutive workgroups go round-robin over the 8 XCDs, so each XCD gets a
// contiguous range of the order (the grid is 8 * per workgroups).
__device__ __forceinline__ int xcd_order(int n_triples) {
    const int per = gridDim.x / 8;
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
    // the same for every lane of the wave: keep it (and all that derives
    // from it) in scalar registers
    const int o = __builtin_amdgcn_readfirstlane((xcd * per + slot) * kWavesPerBlock + (int)threadIdx.x / kWave);
    return o < n_triples ? o : -1;
}

struct Triple {
    int ia, it, ic;     // mesh indices of s, t, u
    long out;           // (su * nf + t): element offset / ns of the output
    double s, t, u, w1p, w2p, w1, w2;
};

__device__ __forceinline__ Triple make_triple(const double* w, int nf, int ia, int it, int ic) {
    Triple T;
    T.ia = ia; T.it = it; T.ic = ic;
    T.out = (su_index(ia, ic) * nf + it);
    T.s = w[ia]; T.t = w[it]; T.u = w[ic];
    // external frequencies from s = w1'+w2', t = w1'-w1, u = w1'-w2 (Eq. 17)
    T.w1p = 0.5 * (T.s + T.t + T.u);
    T.w2p = 0.5 * (T.s - T.t - T.u);
    T.w1 = 0.5 * (T.s - T.t + T.u);
    T.w2 = 0.5 * (T.s + T.t - T.u);
    return T;
}

// Sum the per-group partials (lanes g*ns + p) and write (or add) pair p.
__device__ __forceinline__ void finish_pairs(double* red, int lane, int ns, int G, bool act, double acc_s,
                                             double acc_d, double extra_s, double extra_d, double* ds,
                                             double* dd, bool add) {
    red[lane] = act ? acc_s : 0.0;
    red[kWave + lane] = act ? acc_d : 0.0;
    wave_lds_sync();
    if (lane < ns) {
        double ts = extra_s, td = extra_d;
        for (int gg = 0; gg < G; ++gg) {
            ts += red[gg * ns + lane];
            td += red[kWave + gg * ns + lane];
        }
        if (add) { ds[lane] += ts; dd[lane] += td; }
        else { ds[lane] = ts; dd[lane] = td; }
    }
}

// The per-lane result of one channel body: lanes (g, p) hold partial sums
// for pair p that finish_pairs adds up over the groups g.
struct LanePart {
    double s, d;
};

// s/u channels: lanes (g, q) hold partial sums for the pairs q * kSuPairs + h.
struct SuPart {
    double s[2] = {0.0, 0.0}, d[2] = {0.0, 0.0};
};

// Sum the s/u partials over the groups and write (or add) every pair.
template <class R>
__device__ __forceinline__ void finish_su(double* red, int lane, int ns, const SuPart& v, double* ds, double* dd,
                                          bool add) {
    constexpr int PL = kSuPairs<R>;
    const int np = (ns + PL - 1) / PL, G = kWave / np;
    const bool act = lane / np < G;
#pragma unroll
    for (int h = 0; h < PL; ++h) {
        red[h * kWave + lane] = act ? v.s[h] : 0.0;
        red[(PL + h) * kWave + lane] = act ? v.d[h] : 0.0;
    }
    wave_lds_sync();
    if (lane < ns) {
        const int q = lane / PL, h = lane % PL;
        double ts = 0.0, td = 0.0;
        for (int gg = 0; gg < G; ++gg) {
            ts += red[h * kWave + gg * np + q];
            td += red[(PL + h) * kWave + gg * np + q];
        }
        if (add) { ds[lane] += ts; dd[lane] += td; }
        else { ds[lane] = ts; dd[lane] = td; }
    }
}

// Byte offsets of a lane's two adjacent pairs p0 = 2q, p0 + 1 (FP32): un for
// the unexchanged element p0, sw0 / sw1 for the exchange partners of the two
// pairs; two_loads when the partners are not adjacent (the second pair's
// corners are then read on their own).
struct PairOff2 {
    unsigned un, sw0, sw1;
    bool two_loads;
};

// Interpolation of both vectors (plans Pa, Pb) for the two pairs of a lane:
// a[h] / b[h] = (spin, density) of pair 2q + h.  All eight 16-byte corner
// loads are issued before any arithmetic.
__device__ __forceinline__ void eval_packed_ab2(const PlanT<float>& Pa, const PlanT<float>& Pb,
                                                __amdgpu_buffer_rsrc_t r, const PairOff2& po, float2 (&a)[2],
                                                float2 (&b)[2]) {
    const unsigned qa = Pa.swp ? po.sw0 : po.un, qb = Pb.swp ? po.sw0 : po.un;
    float4 ga[4], gb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        ga[i] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)((unsigned)Pa.off[i] + qa), 0, 0));
#pragma unroll
    for (int i = 0; i < 4; ++i)
        gb[i] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)((unsigned)Pb.off[i] + qb), 0, 0));
    if (po.two_loads) {
        if (Pa.swp)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float2 v = load_corner(r, (unsigned)Pa.off[i] + po.sw1, float());
                ga[i].z = v.x;
                ga[i].w = v.y;
            }
        if (Pb.swp)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float2 v = load_corner(r, (unsigned)Pb.off[i] + po.sw1, float());
                gb[i].z = v.x;
                gb[i].w = v.y;
            }
    }
    float a0 = 0, a1 = 0, a2 = 0, a3 = 0, b0 = 0, b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        a0 = fmaf(Pa.ws[i], ga[i].x, a0);
        a1 = fmaf(Pa.wd[i], ga[i].y, a1);
        a2 = fmaf(Pa.ws[i], ga[i].z, a2);
        a3 = fmaf(Pa.wd[i], ga[i].w, a3);
        b0 = fmaf(Pb.ws[i], gb[i].x, b0);
        b1 = fmaf(Pb.wd[i], gb[i].y, b1);
        b2 = fmaf(Pb.ws[i], gb[i].z, b2);
        b3 = fmaf(Pb.wd[i], gb[i].w, b3);
    }
    a[0] = make_float2(a0, a1);
    a[1] = make_float2(a2, a3);
    b[0] = make_float2(b0, b1);
    b[1] = make_float2(b2, b3);
}

// s channel (CH = 0): A = Gamma(s, w1'-w, w-w2'), B = Gamma(s, w-w1, w-w2),
//   dGs += W (-2 As Bs + As Bd + Ad Bs), dGd += W (3 As Bs + Ad Bd).
// u channel (CH = 2): A = Gamma(w1+w, w-w2', u), B = Gamma(w1'+w, w2-w, u),
//   dGs += W (2 As Bs + As Bd + Ad Bs), dGd += W (3 As Bs + Ad Bd).
// R: precision of the interpolation, products and per-chunk sums (the chunk
// sums are folded by CompSum).  A.w must point at the LDS mesh copy; plan is
// the wave's LDS plan area.
template <int CH, class R>
__device__ __forceinline__ SuPart su_body(const FlowArgs& A, const Shared& sh, PlanT<R>* plan, const Triple& T,
                                          __amdgpu_buffer_rsrc_t rv, int lane) {
    // the chunk's node weights sit in LDS after the plans
    double* wts = reinterpret_cast<double*>(plan + 2 * kPlanChunk);
    constexpr int PL = kSuPairs<R>;
    const int nf = A.nf, ns = A.ns, nq = A.nq;
    const int ia = T.ia, ic = T.ic;
    const int np = (ns + PL - 1) / PL;
    const int G = kWave / np;
    const int g = lane / np, q = lane % np;
    const bool act = g < G;
    const int p0 = PL * q;
    int2 pp{0, 0};
    PairOff2 po{0u, 0u, 0u, false};
    if constexpr (PL == 1) {
        pp = make_int2(kElemBytes<R> * p0, kElemBytes<R> * sh.swap[p0]);
    } else {
        const int s0 = sh.swap[p0];
        const bool second = p0 + 1 < ns;
        const int s1 = second ? sh.swap[p0 + 1] : s0 + 1;
        po = PairOff2{(unsigned)(kElemBytes<R> * p0), (unsigned)(kElemBytes<R> * s0), (unsigned)(kElemBytes<R> * s1),
                      s1 != s0 + 1};
    }
    CompSum<R> sum_s[PL], sum_d[PL];
    const int iv = CH == 0 ? ia : ic;
    const int cnt = A.tab_n[CH * nf + iv];
    const double* tw = A.tab_w + (long)(CH * nf + iv) * nq;
    const double* tg = A.tab_g + (long)(CH * nf + iv) * nq;
    const R sgn = CH == 0 ? R(-2) : R(2);
    const R three = R(3);
    R acc_s[PL], acc_d[PL];
#pragma unroll
    for (int h = 0; h < PL; ++h) acc_s[h] = acc_d[h] = R(0);
    for (int k0 = 0; k0 < cnt; k0 += kPlanChunk) {
        const int kc = min(kPlanChunk, cnt - k0);
        {
            const int j = lane % kPlanChunk, vec = lane / kPlanChunk;
            if (j < kc) {
                const double om = tw[k0 + j];
                // arguments chosen per lane, one plan construction for all
                PlanT<R> P;
                if (CH == 0)
                    make_plan(A.w, nf, ns, T.s, vec == 0 ? T.w1p - om : om - T.w1, vec == 0 ? om - T.w2p : om - T.w2,
                              0, ia, P, &sh.lut);
                else
                    make_plan(A.w, nf, ns, vec == 0 ? T.w1 + om : T.w1p + om, vec == 0 ? om - T.w2p : T.w2 - om, T.u,
                              2, ic, P, &sh.lut);
                to_bytes(P);
                plan[vec * kPlanChunk + j] = P;
                if (vec == 0) wts[j] = tg[k0 + j];
            }
        }
        wave_lds_sync();
        if (act) {
            for (int k = g; k < kc; k += G) {
                const R W = (R)wts[k];
                if constexpr (PL == 1) {
                    R as, ad, bs, bd;
                    eval_packed_ab(plan[k], plan[kPlanChunk + k], rv, pp, as, ad, bs, bd);
                    acc_s[0] = fmr(W, sgn * as * bs + as * bd + ad * bs, acc_s[0]);
                    acc_d[0] = fmr(W, three * as * bs + ad * bd, acc_d[0]);
                } else {
                    float2 a[2], b[2];
                    eval_packed_ab2(plan[k], plan[kPlanChunk + k], rv, po, a, b);
#pragma unroll
                    for (int h = 0; h < PL; ++h) {
                        acc_s[h] = fmr(W, sgn * a[h].x * b[h].x + a[h].x * b[h].y + a[h].y * b[h].x, acc_s[h]);
                        acc_d[h] = fmr(W, three * a[h].x * b[h].x + a[h].y * b[h].y, acc_d[h]);
                    }
                }
            }
        }
        if constexpr (sizeof(R) == 4) {
#pragma unroll
            for (int h = 0; h < PL; ++h) {
                sum_s[h].add(acc_s[h]);
                sum_d[h].add(acc_d[h]);
                acc_s[h] = acc_d[h] = R(0);
            }
        }
        wave_lds_sync();
    }
    SuPart out;
#pragma unroll
    for (int h = 0; h < PL; ++h) {
        if constexpr (sizeof(R) == 8) {
            sum_s[h].s = acc_s[h];
            sum_d[h].s = acc_d[h];
        }
        out.s[h] = act ? sum_s[h].value() : 0.0;
        out.d[h] = act ? sum_d[h].value() : 0.0;
    }
    return out;
}
template <int CH, class R>
static __global__ void __launch_bounds__(kWave * kWavesPerBlock)
k_vertex_su(FlowArgs A, const V2<R>* __restrict__ gv, const int* __restrict__ uo_a,
            const int* __restrict__ uo_c, int n_triples, double* __restrict__ dx) {
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int nf = A.nf, ns = A.ns;
    const Shared sh = load_shared(A, lds_raw, false);
    A.w = sh.w;
    const WaveLds<R> L{ns};
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    unsigned char* base = lds_raw + SharedLds{nf, ns, A.n_terms}.bytes(false) + wid * L.su_bytes();
    PlanT<R>* plan = reinterpret_cast<PlanT<R>*>(base);
    double* red = reinterpret_cast<double*>(base + L.su_bytes() - L.red());
    const int o = xcd_order(n_triples);
    if (o < 0) return;
    const int q = o / nf, it = o % nf;
    const int ia = CH == 0 ? A.su_a[q] : uo_a[q];
    const int ic = CH == 0 ? A.su_c[q] : uo_c[q];
    const Triple T = make_triple(A.w, nf, ia, it, ic);
    const __amdgpu_buffer_rsrc_t rv = vertex_rsrc<R>(gv, (long)n_triples * ns);
    const SuPart r = su_body<CH, R>(A, sh, plan, T, rv, lane);
    const long vsz = (long)n_triples * ns;
    finish_su<R>(red, lane, ns, r, dx + A.nf + T.out * ns, dx + A.nf + vsz + T.out * ns, CH != 0);
}

// t channel:
//   RPA:  -sum_j Gamma_{i1 j}(w1+w, t, w1'-w) Gamma_{j i2}(w+w2', t, w-w2)
//   corr: Gamma_{i1i2}(w1+w, t, w1'-w) Gamma_{i2i2}(w2'+w, w2-w, -t)
//       + Gamma_{i1i1}(w1+w, w-w1', -t) Gamma_{i1i2}(w+w2', t, w-w2)
// The lattice sum is the matrix M = sum_k W_k a_k b_k^T (both strains),
// contracted with the tabulated (ka, kb, count) terms of each output pair.
// M is accumulated either on the matrix cores, in 16x16 tiles taking four
// nodes per step with their operands read from the site vectors in LDS
// (TMatrixCores below says when), or register-blocked 2x4 per lane on the
// vector ALU.  In FP32 the matrix of each plan chunk is folded into a
// compensated sum; the contraction with the terms runs in FP64.  NSP = pair
// count padded to a multiple of 4 (compile-time, so LDS offsets are
// immediates); NB = vector-ALU blocks per lane; NT = tiles per matrix side.
// Nodes per lattice-sum sub-chunk: 8 where one 2x4 register block per lane
// covers the matrix (17 to 20 pairs), else 4 (one matrix-core step, or two
// register blocks per lane), which also keeps the LDS of a workgroup small
// enough for five per CU at up to 16 pairs.
__host__ __device__ constexpr int t_sub(int nsp) { return nsp > 16 && nsp <= 20 ? kSub : kSub / 2; }

template <int NSP>
struct TShape {
    static constexpr int NB = ((NSP / 2) * (NSP / 4) + kWave - 1) / kWave;
    static constexpr int SUB = t_sub(NSP);
    static constexpr int NT = (NSP + 15) / 16;
};

// Lanes of v_mfma_f64_16x16x4f64 and v_mfma_f32_16x16x4f32 (64 lanes):
// operand A(16x4) element (i, k) and B(4x16) element (k, j) sit in lane
// i + 16k resp. j + 16k; result register r of lane l holds D(l / 16 + 4r,
// l % 16) in FP64 and D(4 (l / 16) + r, l % 16) in FP32.
template <class R> using Vec4 = R __attribute__((ext_vector_type(4)));
template <class R>
__device__ __forceinline__ Vec4<R> mfma16x16x4(R a, R b, Vec4<R> c) {
    if constexpr (sizeof(R) == 8) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <class R>
__device__ __forceinline__ int mfma_row(int lane, int r) {
    return sizeof(R) == 8 ? lane / 16 + 4 * r : 4 * (lane / 16) + r;
}
// Matrix cores for the lattice sum: while one tile covers the pairs, and in
// FP64 also beyond 20 pairs, where the vector-ALU blocks need as many
// registers as the four tiles (from 17 to 20 pairs the tiles would cost a
// wave per SIMD; in FP32 every matrix entry carries a compensated sum).
template <class R, int NSP> struct TMatrixCores {
    static constexpr bool on = NSP <= 16 || (sizeof(R) == 8 && NSP > 20);
};

// base: the wave's LDS area (layout WaveLds<R>{ns, SUB}); sh.off / sh.terms
// (and beyond 20 pairs sh.run) must hold the lattice-sum tables.
template <int NSP, class R>
__device__ __forceinline__ LanePart t_body(const FlowArgs& A, const Shared& sh, unsigned char* base,
                                           const Triple& T, __amdgpu_buffer_rsrc_t rv, int lane) {
    constexpr int NB = TShape<NSP>::NB;
    constexpr int SUB = TShape<NSP>::SUB;
    constexpr int NBK = NSP / 4;
    constexpr bool kComp = sizeof(R) == 4;
    const int nf = A.nf, ns = A.ns, nq = A.nq;
    const WaveLds<R> L{ns, SUB};
    TPlan<R>* plan = reinterpret_cast<TPlan<R>*>(base);                           // [2][kTChunk]
    R* ons = reinterpret_cast<R*>(base + L.plans());                                // [5][kTChunk]: on-site, weights
    R* wts = ons + 4 * kTChunk;
    R* vb = reinterpret_cast<R*>(base + L.plans() + L.onsite());                    // [4][SUB][NSP]
    double* mat = reinterpret_cast<double*>(base);                                  // [ns*ns] at the end
    const int it = T.it;
    const double t = T.t;

    const int G = kWave / ns;
    const int g = lane / ns, p = lane % ns;
    const bool act = g < G;
    const int2 pp = make_int2(kElemBytes<R> * p, kElemBytes<R> * sh.swap[p]);
    CompSum<R> sum_s, sum_d;
    const R three = R(3);
    R acc_s = 0, acc_d = 0;

    const int cnt = A.tab_n[1 * nf + it];
    const double* tw = A.tab_w + (long)(1 * nf + it) * nq;
    const double* tg = A.tab_g + (long)(1 * nf + it) * nq;

    constexpr bool kMat = TMatrixCores<R, NSP>::on;
    constexpr int NT = kMat ? TShape<NSP>::NT : 1;
    // padding columns ns .. NSP-1 of the site vectors stay zero
    if constexpr (!kMat)
        for (int i = lane; i < 4 * SUB * NSP; i += kWave)
            if (i % NSP >= ns) vb[i] = R(0);
    Vec4<R> cs[NT][NT], cd[NT][NT];
    CompSum<R> ccs[kMat && kComp ? NT : 1][kMat && kComp ? NT : 1][4],
        ccd[kMat && kComp ? NT : 1][kMat && kComp ? NT : 1][4];
    if constexpr (kMat)
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
            for (int J = 0; J < NT; ++J) { cs[I][J] = Vec4<R>{0, 0, 0, 0}; cd[I][J] = Vec4<R>{0, 0, 0, 0}; }

    // register blocks: block b = lane + 64 r covers rows 2*(b / NBK) .. +1
    // and columns 4*(b % NBK) .. +3
    const int nblocks = ((ns + 1) / 2) * NBK;
    R ms[NB][2][4], md[NB][2][4];
    CompSum<R> cms[kComp ? NB : 1][2][4], cmd[kComp ? NB : 1][2][4];
#pragma unroll
    for (int r = 0; r < NB; ++r)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) { ms[r][i][j] = R(0); md[r][i][j] = R(0); }

    for (int k0 = 0; k0 < cnt; k0 += kTChunk) {
        const int kc = min(kTChunk, cnt - k0);
        {
            // lane (role, j): role 0/1 the site-vector plans a/b of node j,
            // role 2/3 the on-site vertices of the two corrections
            const int j = lane % kTChunk, role = lane / kTChunk;
            if (j < kc) {
                const double om = tw[k0 + j];
                // arguments chosen per lane, one plan construction for all
                const double a0 = role == 0 ? T.w1 + om : (role == 1 ? om + T.w2p : (role == 2 ? T.w2p + om : T.w1 + om));
                const double a1 = role == 0 ? t : (role == 1 ? t : (role == 2 ? T.w2 - om : om - T.w1p));
                const double a2 = role == 0 ? T.w1p - om : (role == 1 ? om - T.w2 : -t);
                TPlan<R> P;
                make_plan(A.w, nf, ns, a0, a1, a2, role < 2 ? 1 : 2, it, P, &sh.lut);
                to_bytes(P);
                if (role < 2) {
                    plan[role * kTChunk + j] = P;
                    if (role == 0) wts[j] = (R)tg[k0 + j];
                } else {
                    R os, od;
                    eval_packed2(P, rv, make_int2(0, 0), os, od);      // on-site pair 0
                    ons[(2 * (role - 2) + 0) * kTChunk + j] = os;
                    ons[(2 * (role - 2) + 1) * kTChunk + j] = od;
                }
            }
        }
        wave_lds_sync();
        for (int s0 = 0; s0 < kc; s0 += SUB) {
            const int sc = min(SUB, kc - s0);
            // site vectors of this sub-chunk for pair p: W*a (rows 0, 1) and b
            // (rows 2, 3); the vertex corrections of pair p use the same ones
            if (act) {
                for (int kk = g; kk < sc; kk += G) {
                    R as, ad, bs, bd;
                    eval_packed_ab(plan[s0 + kk], plan[kTChunk + s0 + kk], rv, pp, as, ad, bs, bd);
                    const R W = wts[s0 + kk];
                    const R was = W * as, wad = W * ad;
                    vb[(0 * SUB + kk) * NSP + p] = was;
                    vb[(1 * SUB + kk) * NSP + p] = wad;
                    vb[(2 * SUB + kk) * NSP + p] = bs;
                    vb[(3 * SUB + kk) * NSP + p] = bd;
                    const R* on = ons + s0 + kk;
                    const R o1s = on[0 * kTChunk], o1d = on[1 * kTChunk];
                    const R o2s = on[2 * kTChunk], o2d = on[3 * kTChunk];
                    acc_s += -was * o1s + was * o1d + W * (-o2s * bs + o2d * bs);
                    acc_d += three * wad * o1s + wad * o1d + W * (three * o2s * bd + o2d * bd);
                }
            }
            wave_lds_sync();
            // lattice-sum matrix: M[ka][kb] += (W a)[ka] b[kb], both strains
            if constexpr (kMat) {
                const int i16 = lane % 16, k4 = lane / 16;
#pragma unroll
                for (int kq = 0; kq < SUB; kq += 4) {
                    if (kq < sc) {
                        const int kk = kq + k4;
                        R xa[2][NT], xb[2][NT];
#pragma unroll
                        for (int I = 0; I < NT; ++I) {
                            const int pr = 16 * I + i16;
                            const bool in = kk < sc && pr < ns;
                            const int o = in ? kk * NSP + pr : 0;
                            xa[0][I] = vb[0 * SUB * NSP + o];
                            xa[1][I] = vb[1 * SUB * NSP + o];
                            xb[0][I] = vb[2 * SUB * NSP + o];
                            xb[1][I] = vb[3 * SUB * NSP + o];
                            if (!in) xa[0][I] = xa[1][I] = xb[0][I] = xb[1][I] = R(0);
                        }
#pragma unroll
                        for (int I = 0; I < NT; ++I)
#pragma unroll
                            for (int J = 0; J < NT; ++J) {
                                cs[I][J] = mfma16x16x4<R>(xa[0][I], xb[0][J], cs[I][J]);
                                cd[I][J] = mfma16x16x4<R>(xa[1][I], xb[1][J], cd[I][J]);
                            }
                    }
                }
            } else
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const int bidx = lane + kWave * r;
                if (bidx < nblocks) {
                    const int ka0 = 2 * (bidx / NBK), kb0 = 4 * (bidx % NBK);
                    const R* va = vb + ka0;
                    const R* vbb = vb + kb0;
#pragma unroll
                    for (int kk = 0; kk < SUB; ++kk) {
                        if (kk < sc) {
                            const V2<R> xs = *reinterpret_cast<const V2<R>*>(va + (0 * SUB + kk) * NSP);
                            const V2<R> xd = *reinterpret_cast<const V2<R>*>(va + (1 * SUB + kk) * NSP);
                            const V4<R> ys = *reinterpret_cast<const V4<R>*>(vbb + (2 * SUB + kk) * NSP);
                            const V4<R> yd = *reinterpret_cast<const V4<R>*>(vbb + (3 * SUB + kk) * NSP);
                            const R a_s[2] = {xs.x, xs.y}, a_d[2] = {xd.x, xd.y};
                            const R b_s[4] = {ys.x, ys.y, ys.z, ys.w}, b_d[4] = {yd.x, yd.y, yd.z, yd.w};
#pragma unroll
                            for (int i = 0; i < 2; ++i)
#pragma unroll
                                for (int j = 0; j < 4; ++j) {
                                    ms[r][i][j] = fmr(a_s[i], b_s[j], ms[r][i][j]);
                                    md[r][i][j] = fmr(a_d[i], b_d[j], md[r][i][j]);
                                }
                        }
                    }
                }
            }
            wave_lds_sync();
        }
        if constexpr (kComp) {
            sum_s.add(acc_s);
            sum_d.add(acc_d);
            acc_s = acc_d = R(0);
            if constexpr (kMat) {
#pragma unroll
                for (int I = 0; I < NT; ++I)
#pragma unroll
                    for (int J = 0; J < NT; ++J) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            ccs[I][J][r].add(cs[I][J][r]);
                            ccd[I][J][r].add(cd[I][J][r]);
                        }
                        cs[I][J] = Vec4<R>{0, 0, 0, 0};
                        cd[I][J] = Vec4<R>{0, 0, 0, 0};
                    }
            } else
#pragma unroll
            for (int r = 0; r < NB; ++r)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        cms[r][i][j].add(ms[r][i][j]);
                        cmd[r][i][j].add(md[r][i][j]);
                        ms[r][i][j] = R(0);
                        md[r][i][j] = R(0);
                    }
        }
    }

    // the matrix strain by strain (reusing the work area), contracted with
    // the tabulated (ka, kb, count) terms of every output pair.  Beyond 20
    // pairs lane l takes run l of the terms (two sums in turn, for two loads
    // in flight; the run sums of a pair are added after both strains);
    // otherwise lanes (g, p) take every G-th term of pair p, whose short
    // lists gain nothing from the extra reduction
    wave_lds_sync();
    if constexpr (!kComp) {
        sum_s.s = acc_s;
        sum_d.s = acc_d;
    }
    double tot_s = sum_s.value(), tot_d = sum_d.value();
    double* part = reinterpret_cast<double*>(base + L.mat());   // [2][kWave]: free until the pairs finish
    for (int strain = 0; strain < 2; ++strain) {
        if constexpr (kMat) {
#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int J = 0; J < NT; ++J)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int ka = 16 * I + mfma_row<R>(lane, r), kb = 16 * J + lane % 16;
                        double v;
                        if constexpr (kComp) v = strain == 0 ? ccs[I][J][r].value() : ccd[I][J][r].value();
                        else v = strain == 0 ? (double)cs[I][J][r] : (double)cd[I][J][r];
                        if (ka < ns && kb < ns) mat[ka * ns + kb] = v;
                    }
        } else
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int bidx = lane + kWave * r;
            if (bidx < nblocks) {
                const int ka0 = 2 * (bidx / NBK), kb0 = 4 * (bidx % NBK);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int ka = ka0 + i, kb = kb0 + j;
                        double v;
                        if constexpr (kComp) v = strain == 0 ? cms[r][i][j].value() : cmd[r][i][j].value();
                        else v = strain == 0 ? (double)ms[r][i][j] : (double)md[r][i][j];
                        if (ka < ns && kb < ns) mat[ka * ns + kb] = v;
                    }
            }
        }
        wave_lds_sync();
        if constexpr (NSP > 20) {
            const int2 run = sh.run[lane];
            double a0 = 0.0, a1 = 0.0;
            int q = run.x;
            for (; q + 1 < run.y; q += 2) {
                const int t0 = sh.terms[q], t1 = sh.terms[q + 1];
                a0 = fma((double)(t0 >> 16), mat[t0 & 0xffff], a0);
                a1 = fma((double)(t1 >> 16), mat[t1 & 0xffff], a1);
            }
            if (q < run.y) {
                const int t0 = sh.terms[q];
                a0 = fma((double)(t0 >> 16), mat[t0 & 0xffff], a0);
            }
            part[strain * kWave + lane] = a0 + a1;
        } else if (act) {
            double acc = 0.0;
            for (int q = sh.off[p] + g; q < sh.off[p + 1]; q += G) {
                const int tq = sh.terms[q];
                acc = fma((double)(tq >> 16), mat[tq & 0xffff], acc);
            }
            if (strain == 0) tot_s = fma(-2.0, acc, tot_s);
            else tot_d = fma(-2.0, acc, tot_d);
        }
        wave_lds_sync();
    }
    if constexpr (NSP > 20) {
        // pair p (lane g = 0) adds its runs in order
        if (act && g == 0) {
            double rs = 0.0, rd = 0.0;
            for (int l = sh.run_off[p]; l < sh.run_off[p + 1]; ++l) {
                rs += part[l];
                rd += part[kWave + l];
            }
            tot_s = fma(-2.0, rs, tot_s);
            tot_d = fma(-2.0, rd, tot_d);
        }
        wave_lds_sync();
    }
    return LanePart{act ? tot_s : 0.0, act ? tot_d : 0.0};
}

// One context, ordered by (t, s, u); adds to dGamma (add != 0) or writes its
// part (add == 0).  Occupancy targets: the
// widest that hold the register blocks without spilling (five waves per SIMD
// up to 16 pairs, four up to 20, three beyond).
template <int NSP, class R>
static __global__ void __launch_bounds__(kWave * kWavesPerBlock)
__attribute__((amdgpu_waves_per_eu(NSP > 20 ? 3 : (NSP > 16 ? 4 : 5))))
k_vertex_t(FlowArgs A, const V2<R>* __restrict__ gv, int n_triples, double* __restrict__ dx, int add) {
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int nf = A.nf, ns = A.ns;
    const Shared sh = load_shared(A, lds_raw, true, NSP > 20);
    A.w = sh.w;
    const WaveLds<R> L{ns, TShape<NSP>::SUB};
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    unsigned char* base = lds_raw + SharedLds{nf, ns, A.n_terms}.bytes(true) + wid * L.bytes();
    double* red = reinterpret_cast<double*>(base + L.mat());                        // [2][64] at the end
    const int o = xcd_order(n_triples);
    if (o < 0) return;
    const int nsu = nf * (nf + 1) / 2;
    const int it = o / nsu, su = o % nsu;
    const Triple T = make_triple(A.w, nf, A.su_a[su], it, A.su_c[su]);
    const __amdgpu_buffer_rsrc_t rv = vertex_rsrc<R>(gv, (long)n_triples * ns);
    const LanePart r = t_body<NSP, R>(A, sh, base, T, rv, lane);
    const long vsz = (long)n_triples * ns;
    finish_pairs(red, lane, ns, kWave / ns, lane / ns < kWave / ns, r.s, r.d, 0.0, 0.0,
                 dx + A.nf + T.out * ns, dx + A.nf + vsz + T.out * ns, add != 0);
}

// The s, u and t channels in one launch (grid 24 * per workgroups).  The
// hardware deals consecutive workgroups round-robin to the 8 XCDs; within an
// XCD the j-th workgroup takes role j mod 3 (s, u, t) and slot j / 3, and a
// role's slots walk its XCD's contiguous range of triples as in the separate
// launches.  The s role writes dx, the u and t roles write du and dt; the
// LDS area is the larger of the two layouts.
template <int NSP, class R>
static __global__ void __launch_bounds__(kWave * kWavesPerBlock)
__attribute__((amdgpu_waves_per_eu(NSP > 20 ? 3 : (NSP > 16 ? 4 : 5))))
k_vertex_stu(FlowArgs A, const V2<R>* __restrict__ gv, const int* __restrict__ uo_a, const int* __restrict__ uo_c,
             int n_triples, double* __restrict__ dx, double* __restrict__ du, double* __restrict__ dt) {
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int nf = A.nf, ns = A.ns;
    const int xcd = blockIdx.x % 8, j = blockIdx.x / 8;
    const int role = __builtin_amdgcn_readfirstlane(j % 3), slot = j / 3;
    const int per = gridDim.x / 24;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const Shared sh = load_shared(A, lds_raw, role == 2, role == 2 && NSP > 20);
    A.w = sh.w;
    const int o = __builtin_amdgcn_readfirstlane((xcd * per + slot) * kWavesPerBlock + wid);
    if (o >= n_triples) return;
    const long vsz = (long)n_triples * ns;
    const __amdgpu_buffer_rsrc_t rv = vertex_rsrc<R>(gv, vsz);
    if (role < 2) {
        const WaveLds<R> L{ns};
        unsigned char* base = lds_raw + SharedLds{nf, ns, A.n_terms}.bytes(false) + wid * L.su_bytes();
        PlanT<R>* plan = reinterpret_cast<PlanT<R>*>(base);
        double* red = reinterpret_cast<double*>(base + L.su_bytes() - L.red());
        const int q = o / nf, it = o % nf;
        if (role == 0) {
            const Triple T = make_triple(A.w, nf, A.su_a[q], it, A.su_c[q]);
            const SuPart r = su_body<0, R>(A, sh, plan, T, rv, lane);
            finish_su<R>(red, lane, ns, r, dx + nf + T.out * ns, dx + nf + vsz + T.out * ns, false);
        } else {
            const Triple T = make_triple(A.w, nf, uo_a[q], it, uo_c[q]);
            const SuPart r = su_body<2, R>(A, sh, plan, T, rv, lane);
            finish_su<R>(red, lane, ns, r, du + nf + T.out * ns, du + nf + vsz + T.out * ns, false);
        }
    } else {
        const WaveLds<R> L{ns, TShape<NSP>::SUB};
        unsigned char* base = lds_raw + SharedLds{nf, ns, A.n_terms}.bytes(true) + wid * L.bytes();
        double* red = reinterpret_cast<double*>(base + L.mat());
        const int nsu = nf * (nf + 1) / 2;
        const int it = o / nsu, su = o % nsu;
        const Triple T = make_triple(A.w, nf, A.su_a[su], it, A.su_c[su]);
        const LanePart r = t_body<NSP, R>(A, sh, base, T, rv, lane);
        finish_pairs(red, lane, ns, kWave / ns, lane / ns < kWave / ns, r.s, r.d, 0.0, 0.0,
                     dt + nf + T.out * ns, dt + nf + vsz + T.out * ns, false);
    }
}

// x[i] = (x[i] + u[i]) + t[i]: the channel parts in the order of the
// separate launches (grid-stride, any grid size).
static __global__ void __launch_bounds__(256)
k_sum_channels(long n, double* __restrict__ x, const double* __restrict__ u, const double* __restrict__ t) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] = (x[i] + u[i]) + t[i];
}

}  // namespace pffrg
