// kernels_adj.h -- vector-Jacobian products (reverse mode) of the flow
// right-hand side and of the correlations, in FP64.
//
// For a cotangent v of d state / d Lambda (layout of the state) these
// kernels compute J^T v, where J is the Jacobian of the right-hand side
// f(Lambda, state) of kernels_flow.h with respect to the state (self-energy
// and both vertex strains).  The forward pieces are recomputed from the
// state (self-energy derivative, node tables); then, in reverse order:
//   1. vertex channels: every evaluation W_k F(A_k, B_k) of an output element
//      sends v * dF/dA to the four corners of A's interpolation plan and
//      v * dF/dB to B's (the transpose of the gather: scattered with FP64
//      atomics), and v * F to the cotangent of the node weight W_k, summed
//      over the triples and pairs sharing the node list (ctg);
//      the t-channel lattice sum sum_q cnt_q a[ka_q] b[kb_q] is transposed
//      through the matrix N = sum_p v(p) C_p of the term counts C_p:
//      cot a = N b, cot b = N^T a;
//   2. node tables: ctg through the weights' dependence on the self-energy
//      (propagators at the nodes) and on its derivative (Katanin term);
//   3. self-energy flow (Eq. 23): its cotangent (v's own sigma part plus
//      step 2) through the vertex values and propagators it reads.
// Every linear interpolation sig(w) = odd_interp(sig, w) is transposed the
// same way (odd_interp_vjp).
#pragma once

#include "kernels_flow.h"
#include "kernels_obs.h"

namespace pffrg {

__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// Transpose of odd_interp: cot[v_i] += (d value / d v_i) c.
__device__ __forceinline__ void odd_interp_vjp(const double* __restrict__ w, int nf, double x, double c,
                                               double* __restrict__ cot) {
    double sg = 1.0;
    if (x < 0.0) { x = -x; sg = -1.0; }
    int i0, i1;
    double f0, f1;
    bracket(w, nf, x, i0, i1, f0, f1);
    if (f0 != 0.0) atomic_add(cot + i0, sg * f0 * c);
    if (f1 != 0.0) atomic_add(cot + i1, sg * f1 * c);
}

// Both strains at a plan's corners for pair element q (already exchanged),
// from the packed (Gs, Gd) copy of the vertex: one 16-byte load per corner.
__device__ __forceinline__ void eval_packed_el(const Plan& P, __amdgpu_buffer_rsrc_t r, int q, double& vs,
                                               double& vd) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double2 g = load_corner(r, (unsigned)(P.off[i] + q) * 16u, double());
        a = fma(P.ws[i], g.x, a);
        b = fma(P.wd[i], g.y, b);
    }
    vs = a;
    vd = b;
}

// Two plans at once, all eight loads issued before any arithmetic.
__device__ __forceinline__ void eval_packed_el2(const Plan& Pa, int qa, const Plan& Pb, int qb,
                                                __amdgpu_buffer_rsrc_t r, double& as, double& ad, double& bs,
                                                double& bd) {
    double2 ga[4], gb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ga[i] = load_corner(r, (unsigned)(Pa.off[i] + qa) * 16u, double());
#pragma unroll
    for (int i = 0; i < 4; ++i) gb[i] = load_corner(r, (unsigned)(Pb.off[i] + qb) * 16u, double());
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        a0 = fma(Pa.ws[i], ga[i].x, a0);
        a1 = fma(Pa.wd[i], ga[i].y, a1);
        b0 = fma(Pb.ws[i], gb[i].x, b0);
        b1 = fma(Pb.wd[i], gb[i].y, b1);
    }
    as = a0; ad = a1; bs = b0; bd = b1;
}

// Corner contributions of one vector pending along a lane's run of nodes.
// Consecutive nodes often interpolate from some of the same corners; their
// contributions are added in registers and each corner is sent (two FP64
// atomics, spin and density) once when the run leaves it.  Unused corners
// (zero weight) take no slot.
struct PendingCorners {
    int e[4];
    double s[4], d[4];
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int i = 0; i < 4; ++i) { e[i] = -1; s[i] = 0.0; d[i] = 0.0; }
    }
    __device__ __forceinline__ void flush(double* __restrict__ cgs, double* __restrict__ cgd) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (e[i] >= 0) {
                atomic_add(cgs + e[i], s[i]);
                atomic_add(cgd + e[i], d[i]);
            }
        clear();
    }
    // The corners of plan P (pair element q, cotangents cs / cd of its spin
    // and density values) replace the pending ones: a pending corner that P
    // also touches is carried into P's slot, the others are sent.
    __device__ __forceinline__ void push(const Plan& P, int q, double cs, double cd, double* __restrict__ cgs,
                                         double* __restrict__ cgd) {
        int n[4];
        double ns[4], nd[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            n[i] = P.ws[i] != 0.0 ? P.off[i] + q : -1;
            ns[i] = P.ws[i] * cs;
            nd[i] = P.wd[i] * cd;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (e[j] < 0) continue;
            bool carried = false;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (!carried && n[i] == e[j]) {
                    ns[i] += s[j];
                    nd[i] += d[j];
                    carried = true;
                }
            if (!carried) {
                atomic_add(cgs + e[j], s[j]);
                atomic_add(cgd + e[j], d[j]);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) { e[i] = n[i]; s[i] = ns[i]; d[i] = nd[i]; }
    }
};

// Transpose of eval_plan for pair index q (already exchanged): the cotangents
// (cs, cd) of the spin and density values go to the plan's corners.
__device__ __forceinline__ void scatter_plan(const Plan& P, double* __restrict__ cgs, double* __restrict__ cgd,
                                             int q, double cs, double cd) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (P.ws[i] != 0.0) {
            atomic_add(cgs + P.off[i] + q, P.ws[i] * cs);
            atomic_add(cgd + P.off[i] + q, P.wd[i] * cd);
        }
    }
}

static __global__ void k_fill(long n, double v, double* __restrict__ p) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

// Sum of the ns values red[g*ns .. g*ns+ns) of group g (one lane per group
// calls it).
__device__ __forceinline__ double group_sum(const double* red, int g, int ns) {
    double s = 0.0;
    for (int i = 0; i < ns; ++i) s += red[g * ns + i];
    return s;
}

// ----------------------------------------------------------- s, u ------

// One wave per triple (as k_vertex_su).  v: cotangent of the state
// derivative; cgs/cgd: cotangent of the vertex strains (accumulated);
// ctg: cotangent of the node weights [3][nf][nq] (accumulated).
constexpr int kAdjWaves = 4;

struct AdjWaveLds {
    __host__ __device__ static constexpr size_t plans() { return (size_t)2 * kPlanChunk * sizeof(Plan); }
    __host__ __device__ static constexpr size_t red() { return (size_t)kPlanChunk * sizeof(double); }
    __host__ __device__ static constexpr size_t bytes() { return ((plans() + red()) + 31) & ~(size_t)31; }
};

// The vertex-channel products scatter into one of kCotCopies copies of the
// vertex cotangent (copies copy_stride doubles apart), which spreads the
// atomic adds that land on one element over several addresses.  Each XCD
// owns kCotCopies / 8 of the copies (the workgroup's XCD is its index mod 8),
// so no copy takes atomic adds from two XCDs, and neighbouring workgroups of
// one XCD, which work on nearby triples and hit the same elements, take
// different ones of its copies (slot within the XCD, index / 8, modulo the
// count).  k_sum_copies adds the copies up.
constexpr int kCotCopies = 32;

__device__ __forceinline__ long cot_copy(long stride) { return (long)((blockIdx.x % 8) * (kCotCopies / 8) + (blockIdx.x / 8) % (kCotCopies / 8)) * stride; }

template <int CH>
static __global__ void __launch_bounds__(kWave * kAdjWaves)
k_vertex_vjp_su(FlowArgs A, const V2<double>* __restrict__ gv,
                const int* __restrict__ uo_a, const int* __restrict__ uo_c, int n_triples,
                const double* __restrict__ v, double* __restrict__ cgs, double* __restrict__ cgd, long copy_stride,
                double* __restrict__ ctg) {
    cgs += cot_copy(copy_stride);
    cgd += cot_copy(copy_stride);
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int nf = A.nf, ns = A.ns, nq = A.nq;
    const Shared sh = load_shared(A, lds_raw, false);
    A.w = sh.w;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    unsigned char* base = lds_raw + SharedLds{nf, ns, A.n_terms}.bytes(false) + wid * AdjWaveLds::bytes();
    Plan* plan = reinterpret_cast<Plan*>(base);
    double* red = reinterpret_cast<double*>(base + AdjWaveLds::plans());
    const int blocks = gridDim.x;
    const int per = blocks / 8;
    const int o = __builtin_amdgcn_readfirstlane(((blockIdx.x % 8) * per + blockIdx.x / 8) * kAdjWaves + wid);
    if (o >= n_triples) return;
    // the opposite order of the forward launch: waves running together
    // work on different slices of the channel, so their scatters rarely hit
    // the same addresses
    const int q = o / nf, it = o % nf;
    const int ia = CH == 2 ? A.su_a[q] : uo_a[q];
    const int ic = CH == 2 ? A.su_c[q] : uo_c[q];
    const Triple T = make_triple(A.w, nf, ia, it, ic);
    const long vsz = (long)n_triples * ns;
    const __amdgpu_buffer_rsrc_t rv = vertex_rsrc<double>(gv, vsz);

    const int G = kWave / ns;
    const int g = lane / ns, p = lane % ns;
    const bool act = g < G;
    const double vs = act ? v[nf + T.out * ns + p] : 0.0;
    const double vd = act ? v[nf + vsz + T.out * ns + p] : 0.0;
    const int iv = CH == 0 ? ia : ic;
    const int cnt = A.tab_n[CH * nf + iv];
    const double* tw = A.tab_w + (long)(CH * nf + iv) * nq;
    const double* tg = A.tab_g + (long)(CH * nf + iv) * nq;
    double* ct = ctg + (long)(CH * nf + iv) * nq;
    const double sgn = CH == 0 ? -2.0 : 2.0;
    for (int k0 = 0; k0 < cnt; k0 += kPlanChunk) {
        const int kc = min(kPlanChunk, cnt - k0);
        {
            const int j = lane % kPlanChunk, vec = lane / kPlanChunk;
            if (j < kc) {
                const double om = tw[k0 + j];
                Plan P;
                if (CH == 0) {
                    if (vec == 0) make_plan(A.w, nf, ns, T.s, T.w1p - om, om - T.w2p, 0, ia, P, &sh.lut);
                    else make_plan(A.w, nf, ns, T.s, om - T.w1, om - T.w2, 0, ia, P, &sh.lut);
                } else {
                    if (vec == 0) make_plan(A.w, nf, ns, T.w1 + om, om - T.w2p, T.u, 2, ic, P, &sh.lut);
                    else make_plan(A.w, nf, ns, T.w1p + om, T.w2 - om, T.u, 2, ic, P, &sh.lut);
                }
                plan[vec * kPlanChunk + j] = P;
            }
            if (lane < kPlanChunk) red[lane] = 0.0;
        }
        wave_lds_sync();
        // lanes of group g walk a contiguous run of the chunk's nodes
        PendingCorners pa, pb;
        pa.clear();
        pb.clear();
        const int kb = (g * kc) / G, ke = ((g + 1) * kc) / G;
        for (int k = kb; k < ke; ++k) {
            if (act) {
                const Plan& Pa = plan[k];
                const Plan& Pb = plan[kPlanChunk + k];
                const int qa = Pa.swp ? sh.swap[p] : p, qb = Pb.swp ? sh.swap[p] : p;
                double as, ad, bs, bd;
                eval_packed_el2(Pa, qa, Pb, qb, rv, as, ad, bs, bd);
                const double W = tg[k0 + k];
                atomicAdd(red + k, vs * (sgn * as * bs + as * bd + ad * bs) + vd * (3.0 * as * bs + ad * bd));
                const double cas = W * (vs * (sgn * bs + bd) + vd * 3.0 * bs);
                const double cad = W * (vs * bs + vd * bd);
                const double cbs = W * (vs * (sgn * as + ad) + vd * 3.0 * as);
                const double cbd = W * (vs * as + vd * ad);
                pa.push(Pa, qa, cas, cad, cgs, cgd);
                pb.push(Pb, qb, cbs, cbd, cgs, cgd);
            }
        }
        if (act) {
            pa.flush(cgs, cgd);
            pb.flush(cgs, cgd);
        }
        wave_lds_sync();
        if (lane < kc) atomic_add(ct + k0 + lane, red[lane]);     // node weights' cotangent (LDS ds_add_f64 above)
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------- t ----

// Per-wave LDS of the t-channel product, one wave per workgroup; plans are
// built kAdjTChunk nodes at a time, one plan per lane (4 per node).
constexpr int kAdjTChunk = kWave / 4;
constexpr int kAdjTSub = kAdjTChunk;     // nodes whose site vectors are gathered at once
struct AdjTLds {
    int ns;
    __host__ __device__ size_t plans() const { return (size_t)4 * kAdjTChunk * sizeof(Plan); }   // Pa Pb Q1 Q2
    __host__ __device__ size_t ons() const { return (size_t)4 * kAdjTChunk * sizeof(double); }
    __host__ __device__ size_t vb() const { return (size_t)4 * kAdjTSub * ns * sizeof(double); }
    __host__ __device__ size_t nmat() const { return (size_t)2 * ns * ns * sizeof(double); }
    __host__ __device__ size_t vin() const { return (size_t)2 * ns * sizeof(double); }
    __host__ __device__ size_t red() const { return (size_t)5 * kAdjTChunk * sizeof(double); }
    __host__ __device__ size_t bytes() const {
        return ((plans() + ons() + vb() + nmat() + vin() + red()) + 31) & ~(size_t)31;
    }
};

// rpat_off[ns*ns + 1], rpat_ent[n_terms]: the lattice-sum terms grouped by
// (ka, kb), entry = p | (count << 16) (the transpose of the per-output table).
static __global__ void __launch_bounds__(kWave)
k_vertex_vjp_t(FlowArgs A, const V2<double>* __restrict__ gv, int n_triples, const int* __restrict__ rpat_off,
               const int* __restrict__ rpat_ent, const double* __restrict__ v, double* __restrict__ cgs,
               double* __restrict__ cgd, long copy_stride, double* __restrict__ ctg) {
    cgs += cot_copy(copy_stride);
    cgd += cot_copy(copy_stride);
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int nf = A.nf, ns = A.ns, nq = A.nq;
    const Shared sh = load_shared(A, lds_raw, false);
    A.w = sh.w;
    const int lane = threadIdx.x;
    const AdjTLds L{ns};
    unsigned char* base = lds_raw + SharedLds{nf, ns, A.n_terms}.bytes(false);
    Plan* plan = reinterpret_cast<Plan*>(base);                                          // [4][kAdjTChunk]
    double* ons = reinterpret_cast<double*>(base + L.plans());                           // [4][kAdjTChunk]
    double* vb = reinterpret_cast<double*>(base + L.plans() + L.ons());                  // [4][kAdjTSub][ns]
    double* nm = reinterpret_cast<double*>(base + L.plans() + L.ons() + L.vb());         // [2][ns*ns]
    double* vin = nm + 2 * ns * ns;                                                      // [2][ns]
    double* red = vin + 2 * ns;                                                          // [5][kAdjTChunk]
    const int per = gridDim.x / 8;
    const int o = __builtin_amdgcn_readfirstlane((int)((blockIdx.x % 8) * per + blockIdx.x / 8));
    if (o >= n_triples) return;
    // (s, u, t) order, the opposite of the forward t launch (see k_vertex_vjp_su)
    const int su = o / nf, it = o % nf;
    const Triple T = make_triple(A.w, nf, A.su_a[su], it, A.su_c[su]);
    const double t = T.t;
    const long vsz = (long)n_triples * ns;
    const __amdgpu_buffer_rsrc_t rv = vertex_rsrc<double>(gv, vsz);

    for (int i = lane; i < ns; i += kWave) {
        vin[i] = v[nf + T.out * ns + i];
        vin[ns + i] = v[nf + vsz + T.out * ns + i];
    }
    wave_lds_sync();
    // N[ka][kb] = sum over outputs p of v(p) * count of (ka, kb) in p's terms
    for (int e = lane; e < ns * ns; e += kWave) {
        double a = 0.0, b = 0.0;
        for (int qq = rpat_off[e]; qq < rpat_off[e + 1]; ++qq) {
            const int en = rpat_ent[qq];
            const double c = (double)(en >> 16);
            a = fma(c, vin[en & 0xffff], a);
            b = fma(c, vin[ns + (en & 0xffff)], b);
        }
        nm[e] = a;
        nm[ns * ns + e] = b;
    }
    const double* nsm = nm;
    const double* ndm = nm + ns * ns;

    const int G = kWave / ns;
    const int g = lane / ns, p = lane % ns;
    const bool act = g < G;
    const double vs = act ? vin[p] : 0.0;
    const double vd = act ? vin[ns + p] : 0.0;
    const int cnt = A.tab_n[1 * nf + it];
    const double* tw = A.tab_w + (long)(1 * nf + it) * nq;
    const double* tg = A.tab_g + (long)(1 * nf + it) * nq;
    double* ct = ctg + (long)(1 * nf + it) * nq;

    for (int k0 = 0; k0 < cnt; k0 += kAdjTChunk) {
        const int kc = min(kAdjTChunk, cnt - k0);
        wave_lds_sync();
        {
            // lane (role, j): role 0/1 the site-vector plans a/b of node j,
            // role 2/3 the on-site plans of the two corrections (kAdjTChunk = 16)
            const int j = lane % kAdjTChunk, role = lane / kAdjTChunk;
            if (j < kc) {
                const double om = tw[k0 + j];
                const double a0 = role == 0 ? T.w1 + om : (role == 1 ? om + T.w2p : (role == 2 ? T.w2p + om : T.w1 + om));
                const double a1 = role == 0 ? t : (role == 1 ? t : (role == 2 ? T.w2 - om : om - T.w1p));
                const double a2 = role == 0 ? T.w1p - om : (role == 1 ? om - T.w2 : -t);
                Plan P;
                make_plan(A.w, nf, ns, a0, a1, a2, role < 2 ? 1 : 2, it, P, &sh.lut);
                plan[role * kAdjTChunk + j] = P;
                if (role >= 2) {
                    double os, od;
                    eval_packed_el(P, rv, P.swp ? sh.swap[0] : 0, os, od);
                    ons[(2 * (role - 2) + 0) * kAdjTChunk + j] = os;
                    ons[(2 * (role - 2) + 1) * kAdjTChunk + j] = od;
                }
            }
            for (int i = lane; i < 5 * kAdjTChunk; i += kWave) red[i] = 0.0;
        }
        wave_lds_sync();
        for (int s0 = 0; s0 < kc; s0 += kAdjTSub) {
            const int sc = min(kAdjTSub, kc - s0);
            if (act) {
                for (int kk = g; kk < sc; kk += G) {
                    double as, ad, bs, bd;
                    const Plan& Pa = plan[s0 + kk];
                    const Plan& Pb = plan[kAdjTChunk + s0 + kk];
                    eval_packed_el2(Pa, Pa.swp ? sh.swap[p] : p, Pb, Pb.swp ? sh.swap[p] : p, rv, as, ad, bs, bd);
                    vb[(0 * kAdjTSub + kk) * ns + p] = as;
                    vb[(1 * kAdjTSub + kk) * ns + p] = ad;
                    vb[(2 * kAdjTSub + kk) * ns + p] = bs;
                    vb[(3 * kAdjTSub + kk) * ns + p] = bd;
                }
            }
            wave_lds_sync();
            if (act) {
                // lanes of group g walk a contiguous run of the sub-chunk's
                // nodes, merging the corners consecutive nodes share
                PendingCorners pa, pb;
                pa.clear();
                pb.clear();
                for (int kk = (g * sc) / G; kk < ((g + 1) * sc) / G; ++kk) {
                    const int k = s0 + kk;
                    const double W = tg[k0 + k];
                    const double o1s = ons[0 * kAdjTChunk + k], o1d = ons[1 * kAdjTChunk + k];
                    const double o2s = ons[2 * kAdjTChunk + k], o2d = ons[3 * kAdjTChunk + k];
                    const double* ra = vb + (0 * kAdjTSub + kk) * ns;
                    const double* rad = vb + (1 * kAdjTSub + kk) * ns;
                    const double* rb = vb + (2 * kAdjTSub + kk) * ns;
                    const double* rbd = vb + (3 * kAdjTSub + kk) * ns;
                    const double as = ra[p], ad = rad[p], bs = rb[p], bd = rbd[p];
                    // (N b)[p] and (N^T a)[p] for both strains
                    double nbs = 0.0, nbd = 0.0, nas = 0.0, nad = 0.0;
                    for (int j = 0; j < ns; ++j) {
                        nbs = fma(nsm[p * ns + j], rb[j], nbs);
                        nbd = fma(ndm[p * ns + j], rbd[j], nbd);
                        nas = fma(nsm[j * ns + p], ra[j], nas);
                        nad = fma(ndm[j * ns + p], rad[j], nad);
                    }
                    const double cs = -as * o1s + as * o1d - o2s * bs + o2d * bs;
                    const double cd = 3.0 * ad * o1s + ad * o1d + 3.0 * o2s * bd + o2d * bd;
                    const double cas = W * (vs * (o1d - o1s) - 2.0 * nbs);
                    const double cad = W * (vd * (3.0 * o1s + o1d) - 2.0 * nbd);
                    const double cbs = W * (vs * (o2d - o2s) - 2.0 * nas);
                    const double cbd = W * (vd * (3.0 * o2s + o2d) - 2.0 * nad);
                    const Plan& Pa = plan[k];
                    const Plan& Pb = plan[kAdjTChunk + k];
                    pa.push(Pa, Pa.swp ? sh.swap[p] : p, cas, cad, cgs, cgd);
                    pb.push(Pb, Pb.swp ? sh.swap[p] : p, cbs, cbd, cgs, cgd);
                    // per-node sums over the pairs (LDS ds_add_f64)
                    atomicAdd(red + k, vs * cs + vd * cd - 2.0 * (as * nbs + ad * nbd));
                    atomicAdd(red + kAdjTChunk + k, W * (-vs * as + 3.0 * vd * ad));
                    atomicAdd(red + 2 * kAdjTChunk + k, W * (vs * as + vd * ad));
                    atomicAdd(red + 3 * kAdjTChunk + k, W * (-vs * bs + 3.0 * vd * bd));
                    atomicAdd(red + 4 * kAdjTChunk + k, W * (vs * bs + vd * bd));
                }
                pa.flush(cgs, cgd);
                pb.flush(cgs, cgd);
            }
            wave_lds_sync();
        }
        // flush the chunk: node weights and the two on-site vertices (pair 0)
        if (lane < kc) {
            atomic_add(ct + k0 + lane, red[lane]);
            scatter_plan(plan[2 * kAdjTChunk + lane], cgs, cgd, 0, red[kAdjTChunk + lane], red[2 * kAdjTChunk + lane]);
            scatter_plan(plan[3 * kAdjTChunk + lane], cgs, cgd, 0, red[3 * kAdjTChunk + lane],
                         red[4 * kAdjTChunk + lane]);
        }
    }
}

// ------------------------------------------------------ node tables ----

// Reverse of TableWriter for one node list: ctg -> cot_sig, cot_dsig.
struct TableVjp {
    const double* w;
    int nf;
    const double* sig;
    const double* dsig;
    const double* ctg;
    double* cot_sig;
    double* cot_dsig;
    __device__ __forceinline__ void delta(int n, double, double xx, double y, double th) {
        const double c = ctg[n];
        if (c == 0.0) return;
        const double st = 1.0 / (xx - odd_interp(w, nf, sig, xx));
        const double gy = 1.0 / (y - odd_interp(w, nf, sig, y));
        const double tgv = -st * th * gy * kInvTwoPi;
        odd_interp_vjp(w, nf, xx, c * tgv * st, cot_sig);
        odd_interp_vjp(w, nf, y, c * tgv * gy, cot_sig);
    }
    __device__ __forceinline__ void kat(int n, double cur, double pp, double wt) {
        const double c = ctg[n] * wt * kInvTwoPi;
        if (c == 0.0) return;
        const double gw = 1.0 / (cur - odd_interp(w, nf, sig, cur));
        const double gp = 1.0 / (pp - odd_interp(w, nf, sig, pp));
        const double dp = odd_interp(w, nf, dsig, pp), dc = odd_interp(w, nf, dsig, cur);
        odd_interp_vjp(w, nf, pp, c * gw * gp * gp, cot_dsig);
        odd_interp_vjp(w, nf, cur, c * gp * gw * gw, cot_dsig);
        odd_interp_vjp(w, nf, cur, c * (gw * gw * gp * gp * dp + 2.0 * gp * gw * gw * gw * dc), cot_sig);
        odd_interp_vjp(w, nf, pp, c * (2.0 * gw * gp * gp * gp * dp + gp * gp * gw * gw * dc), cot_sig);
    }
    __device__ __forceinline__ void done(int, int) {}
};

// one wave per (channel, nu)
static __global__ void __launch_bounds__(kWave)
k_tables_vjp(FlowArgs A, double lam, const double* __restrict__ x, const double* __restrict__ dsig,
             const double* __restrict__ ctg, double* __restrict__ cot_sig, double* __restrict__ cot_dsig) {
    const int id = blockIdx.x;
    TableVjp vj{A.w, A.nf, x, dsig, ctg + (long)id * A.nq, cot_sig, cot_dsig};
    walk_nodes(A, lam, id, threadIdx.x, vj);
}

// ------------------------------------------------------- self-energy ----

// Reverse of sigma_body: cdsig[n] is the cotangent of d sig(w_n)/d Lambda.
static __global__ void __launch_bounds__(kWave)
k_sigma_vjp(FlowArgs A, double lam, const double* __restrict__ x, long nv, const double* __restrict__ cdsig,
            double* __restrict__ cgs, double* __restrict__ cgd, double* __restrict__ cot_sig) {
    const int n = blockIdx.x, lane = threadIdx.x;
    const double cn = cdsig[n];
    if (cn == 0.0) return;
    const double wn = A.w[n];
    const double* gs = x + A.nf;
    const double* gd = gs + nv;
    for (int sx = 0; sx < 2; ++sx) {
        const double xx = sx == 0 ? lam : -lam;
        Plan P;
        make_plan(A.w, A.nf, A.ns, wn + xx, 0.0, wn - xx, 1, 0, P);
        double f = 0.0;
        for (int r = lane; r < A.ns; r += kWave) {
            double vs, vd;
            eval_plan(P, gs, gd, A.swap, r, vs, vd);
            f = fma(2.0 * (double)A.mult[r], vd, f);
        }
        f = wave_sum(f);
        Plan Q;
        make_plan(A.w, A.nf, A.ns, wn + xx, xx - wn, 0.0, 2, 0, Q);
        double os, od;
        eval_plan(Q, gs, gd, A.swap, 0, os, od);
        f -= 3.0 * os + od;
        const double sv = 1.0 / (xx - odd_interp(A.w, A.nf, x, xx));
        const double c = cn * sv * kInvTwoPi;
        for (int r = lane; r < A.ns; r += kWave)
            scatter_plan(P, cgs, cgd, P.swp ? A.swap[r] : r, 0.0, 2.0 * (double)A.mult[r] * c);
        if (lane == 0) {
            scatter_plan(Q, cgs, cgd, 0, -3.0 * c, -c);
            odd_interp_vjp(A.w, A.nf, xx, cn * f * sv * sv * kInvTwoPi, cot_sig);
        }
    }
}

// ------------------------------------------------------ correlations ----

// Reverse of k_chi_pairs: cchi[p], cchi[ns + p] are the cotangents of
// chi^{zz}_p, chi^{00}_p; one workgroup per pair.  cg2[i] accumulates the
// cotangent of g^2 at correlation node i.
static __global__ void __launch_bounds__(kChiThreads)
k_chi_pairs_vjp(const double* __restrict__ w, int nf, int ns, const int* __restrict__ swap,
                const double* __restrict__ x, const double* __restrict__ cw, const double* __restrict__ cq,
                const double* __restrict__ cg2, const int* __restrict__ cn, const double* __restrict__ cchi,
                double* __restrict__ cgs, double* __restrict__ cgd, double* __restrict__ cot_g2) {
    const int p = blockIdx.x, tid = threadIdx.x;
    const int n = *cn;
    const long vsz = (long)nf * (nf + 1) / 2 * nf * ns;
    const double* gs = x + nf;
    const double* gd = gs + vsz;
    const double pref = 1.0 / (16.0 * M_PI * M_PI);
    const double cz = cchi[p], cd = cchi[ns + p];
    if (cz == 0.0 && cd == 0.0) return;
    for (int e = tid; e < n * n; e += kChiThreads) {
        const int i = e / n, j = e % n;
        const double w1 = cw[i], w2 = cw[j];
        const double qq = cq[i] * cq[j];
        const double f = qq * cg2[i] * cg2[j];
        Plan P;
        make_plan(w, nf, ns, w1 + w2, 0.0, w1 - w2, 1, 0, P);
        double vs, vd;
        eval_plan(P, gs, gd, swap, p, vs, vd);
        double tz = 4.0 * vs, td = 4.0 * vd;
        scatter_plan(P, cgs, cgd, P.swp ? swap[p] : p, -pref * f * 4.0 * cz, -pref * f * 4.0 * cd);
        if (p == 0) {
            Plan Q;
            make_plan(w, nf, ns, w1 + w2, w2 - w1, 0.0, 2, 0, Q);
            double es, ed;
            eval_plan(Q, gs, gd, swap, 0, es, ed);
            tz += 2.0 * es - 2.0 * ed;
            td -= 6.0 * es + 2.0 * ed;
            scatter_plan(Q, cgs, cgd, 0, -pref * f * (2.0 * cz - 6.0 * cd), -pref * f * (-2.0 * cz - 2.0 * cd));
        }
        const double val = -pref * qq * (cz * tz + cd * td);
        atomic_add(cot_g2 + i, val * cg2[j]);
        atomic_add(cot_g2 + j, val * cg2[i]);
    }
    if (p == 0)
        for (int i = tid; i < n; i += kChiThreads) atomic_add(cot_g2 + i, (cz + cd) * cq[i] * 0.5 * kInvTwoPi);
}

// cot_g2 -> cot_sig (g^2 = 1/(w - sig(w))^2, d g^2 / d sig(w) = 2 g^3); one thread.
static __global__ void k_chi_nodes_vjp(const double* __restrict__ w, int nf, const double* __restrict__ x,
                                       const double* __restrict__ cw, const int* __restrict__ cn,
                                       const double* __restrict__ cot_g2, double* __restrict__ cot_sig) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int i = 0; i < *cn; ++i) {
        const double g = 1.0 / (cw[i] - odd_interp(w, nf, x, cw[i]));
        odd_interp_vjp(w, nf, cw[i], cot_g2[i] * 2.0 * g * g * g, cot_sig);
    }
}

// Reverse of k_chi_k: cchi[pair] += (3 / nb) sum_q ck[q] cos(k_q . dr) for
// every (basis, site) term; one thread per term.
static __global__ void k_chi_k_vjp(int nterm, const int* __restrict__ pair, const double* __restrict__ dr,
                                   double inv_nb, int nk, const double* __restrict__ kp,
                                   const double* __restrict__ ck, double* __restrict__ cchi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nterm) return;
    double acc = 0.0;
    for (int q = 0; q < nk; ++q) {
        const double ph = kp[3 * q] * dr[3 * i] + kp[3 * q + 1] * dr[3 * i + 1] + kp[3 * q + 2] * dr[3 * i + 2];
        acc = fma(cos(ph), ck[q], acc);
    }
    atomic_add(cchi + pair[i], 3.0 * inv_nb * acc);
}

// d/d coupling_p of a function of the initial state (Gs = coupling / 4 at
// every frequency): 0.25 * sum over the frequencies of the cotangent of Gs_p.
static __global__ void __launch_bounds__(256)
k_coupling_grad(long n_el, int ns, const double* __restrict__ cgs, double* __restrict__ out) {
    __shared__ double red[256];
    const int p = blockIdx.x;
    double a = 0.0;
    for (long e = threadIdx.x; e < n_el; e += blockDim.x) a += cgs[e * ns + p];
    red[threadIdx.x] = a;
    __syncthreads();
    for (unsigned st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[p] = 0.25 * red[0];
}

// y[i] += sum over the copies of c[copy * stride + i], i < n.
static __global__ void k_sum_copies(long n, long stride, const double* __restrict__ c, double* __restrict__ y) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double acc = y[i];
#pragma unroll
        for (int k = 0; k < kCotCopies; ++k) acc += c[k * stride + i];
        y[i] = acc;
    }
}

// y += alpha * a (elementwise).
static __global__ void k_axpy(long n, double alpha, const double* __restrict__ a, double* __restrict__ y) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] = fma(alpha, a[i], y[i]);
}

}  // namespace pffrg
