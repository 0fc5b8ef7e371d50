// kernels_flow.h -- HIP kernels of the SU(2) pf-FRG right-hand side.
//
// One right-hand side (arXiv:2109.13317, Sec. 3) is three launches:
//   k_sigma_rhs     d sig/d Lambda on the mesh (Eq. 23): the single-scale
//                   propagator pins the internal frequency to +-Lambda;
//   k_node_tables   per channel X in {s,t,u} and transfer frequency index nu,
//                   the evaluation points w_k of the channel's frequency
//                   integral and their weights W_k (delta points of S and
//                   trapezoid nodes of the Katanin term, Eq. 13), so that
//                   channel integral = sum_k W_k F_X(w_k);
//   k_vertex_rhs    one workgroup per output triple (s,t,u): the three channel
//                   sums over their nodes for every pair, the particle-hole
//                   lattice sum in GEMM form (M = sum_k W_k a_k b_k^T per
//                   triple, then the tabulated (ka,kb) terms of each pair).
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
    const int* su_a;        // [nf(nf+1)/2] s-index of each (s,u) wedge entry
    const int* su_c;        //              u-index
    int* tab_n;             // [3*nf] node counts
    double* tab_w;          // [3*nf*nq] node frequencies
    double* tab_g;          // [3*nf*nq] node weights
};

// ------------------------------------------------------------ self-energy -

// d sig/d Lambda (w_n) = (1/2pi) sum_{x=+-Lambda} F(w_n, x) / (x - sig(x)),
// F = 2 sum_r mult_r Gd_r(w+x, 0, w-x) - 3 Gs_0(w+x, x-w, 0) - Gd_0(w+x, x-w, 0).
__global__ void k_sigma_rhs(FlowArgs A, double lam, const double* __restrict__ x,
                            double* __restrict__ dsig) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= A.nf) return;
    const double* sig = x;
    const double* gs = x + A.nf;
    const double* gd = gs + (long)A.nf * (A.nf + 1) / 2 * A.nf * A.ns;
    const double wn = A.w[n];
    double acc = 0.0;
    for (int sx = 0; sx < 2; ++sx) {
        const double xx = sx == 0 ? lam : -lam;
        Plan P, Q;
        make_plan(A.w, A.nf, A.ns, wn + xx, 0.0, wn - xx, P);
        double f = 0.0;
        for (int r = 0; r < A.ns; ++r) {
            double vs, vd;
            eval_plan(P, gs, gd, A.swap, r, vs, vd);
            f = fma(2.0 * (double)A.mult[r], vd, f);
        }
        make_plan(A.w, A.nf, A.ns, wn + xx, xx - wn, 0.0, Q);
        double os, od;
        eval_plan(Q, gs, gd, A.swap, 0, os, od);
        f -= 3.0 * os + od;
        acc += f / (xx - odd_interp(A.w, A.nf, sig, xx));
    }
    dsig[n] = acc * kInvTwoPi;
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

__global__ void k_node_tables(FlowArgs A, double lam, const double* __restrict__ x,
                              const double* __restrict__ dsig) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= 3 * A.nf) return;
    const int ch = id / A.nf, iv = id % A.nf;
    const double nu = A.w[iv];
    const double* sig = x;
    double* tw = A.tab_w + (long)id * A.nq;
    double* tg = A.tab_g + (long)id * A.nq;
    int n = 0;

    // delta parts: the S in Skat(partner(w)) puts w at partner^-1(x); the S in
    // Skat(w) puts w at x.  Weight -G(.) / (x - sig(x)) / (2 pi) in real form.
    for (int sx = 0; sx < 2; ++sx) {
        const double xx = sx == 0 ? lam : -lam;
        const double st = 1.0 / (xx - odd_interp(A.w, A.nf, sig, xx));
        const double winv = ch == 0 ? nu - xx : (ch == 1 ? xx + nu : xx - nu);
        const double pxx = partner(ch, nu, xx);
        double g1 = theta_half(winv, lam);
        double g2 = theta_half(pxx, lam);
        if (g1 != 0.0) {
            g1 /= winv - odd_interp(A.w, A.nf, sig, winv);
            tw[n] = winv; tg[n] = -st * g1 * kInvTwoPi; ++n;
        }
        if (g2 != 0.0) {
            g2 /= pxx - odd_interp(A.w, A.nf, sig, pxx);
            tw[n] = xx; tg[n] = -st * g2 * kInvTwoPi; ++n;
        }
    }

    // Katanin part: trapezoid over the pieces of
    // D = [-wmax, wmax] \ (-lam, lam) \ (c - lam, c + lam), c = zero of the
    // partner; nodes are the piece ends and the mesh points +-w_n inside.
    const double c = ch == 0 ? nu : (ch == 1 ? nu : -nu);
    const double wmax = A.w[A.nf - 1];
    const double e0 = c - lam, e1 = c + lam;
    const double a0[2] = {-wmax, lam}, b0[2] = {-lam, wmax};
    for (int ip = 0; ip < 2; ++ip) {
        const double a = a0[ip], b = b0[ip];
        if (!(a < b)) continue;
        const double lo2[2] = {a, a > e1 ? a : e1};
        const double hi2[2] = {b < e0 ? b : e0, b};
        for (int q = 0; q < 2; ++q) {
            const double lo = lo2[q], hi = hi2[q];
            if (!(lo < hi)) continue;
            // nodes: lo, mesh points +-w_n strictly inside (ascending), hi
            const int first = n;
            tw[n++] = lo;
            for (int i = 0; i < 2 * A.nf; ++i) {
                const double v = i < A.nf ? -A.w[A.nf - 1 - i] : A.w[i - A.nf];
                if (v > lo && v < hi) tw[n++] = v;
            }
            tw[n++] = hi;
            for (int i = first; i < n; ++i) {
                const double cur = tw[i];
                const double wl = i > first ? 0.5 * (cur - tw[i - 1]) : 0.0;
                const double wr = i + 1 < n ? 0.5 * (tw[i + 1] - cur) : 0.0;
                const double pp = partner(ch, nu, cur);
                const double gw = 1.0 / (cur - odd_interp(A.w, A.nf, sig, cur));
                const double gp = 1.0 / (pp - odd_interp(A.w, A.nf, sig, pp));
                const double kat = gw * gp * gp * odd_interp(A.w, A.nf, dsig, pp)
                                 + gp * gw * gw * odd_interp(A.w, A.nf, dsig, cur);
                tg[i] = (wl + wr) * kat * kInvTwoPi;
            }
        }
    }
    A.tab_n[id] = n;
}

// ------------------------------------------------------------- vertex RHS -

constexpr int kThreads = 256;
constexpr int kChunk = 8;      // nodes per chunk of the particle-hole lattice sum

// LDS layout of k_vertex_rhs, in bytes; see vertex_rhs_lds_bytes().
struct VertexLds {
    int nq, ns;
    __host__ __device__ size_t plans() const { return (size_t)2 * nq * sizeof(Plan); }
    __host__ __device__ size_t onsite() const { return (size_t)4 * nq * sizeof(double); }
    __host__ __device__ size_t vchunk() const { return (size_t)4 * kChunk * ns * sizeof(double); }
    __host__ __device__ size_t mat() const { return (size_t)2 * ns * ns * sizeof(double); }
    __host__ __device__ size_t red() const { return (size_t)2 * kThreads * sizeof(double); }
    __host__ __device__ size_t total() const { return plans() + onsite() + vchunk() + mat() + red(); }
};

__global__ void __launch_bounds__(kThreads)
k_vertex_rhs(FlowArgs A, const double* __restrict__ x, double* __restrict__ dx) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const VertexLds L{A.nq, A.ns};
    Plan* plan = reinterpret_cast<Plan*>(lds_raw);
    double* onsite = reinterpret_cast<double*>(lds_raw + L.plans());
    double* vch = reinterpret_cast<double*>(lds_raw + L.plans() + L.onsite());
    double* mat = reinterpret_cast<double*>(lds_raw + L.plans() + L.onsite() + L.vchunk());
    double* red = reinterpret_cast<double*>(lds_raw + L.plans() + L.onsite() + L.vchunk() + L.mat());

    const int nf = A.nf, ns = A.ns, nq = A.nq;
    const long vsz = (long)nf * (nf + 1) / 2 * nf * ns;
    const double* gs = x + nf;
    const double* gd = gs + vsz;
    const int tid = threadIdx.x;
    const int tau = blockIdx.x;
    const int su = tau / nf, it = tau % nf;
    const int ia = A.su_a[su], ic = A.su_c[su];
    const double s = A.w[ia], t = A.w[it], u = A.w[ic];
    // external frequencies from s = w1'+w2', t = w1'-w1, u = w1'-w2 (Eq. 17)
    const double w1p = 0.5 * (s + t + u), w2p = 0.5 * (s - t - u);
    const double w1 = 0.5 * (s - t + u), w2 = 0.5 * (s + t - u);

    // (g, p) decomposition for per-pair accumulation: G groups of ns lanes
    const int G = kThreads / ns;
    const int g = tid / ns, p = tid % ns;
    const bool act = g < G;
    double acc_s = 0.0, acc_d = 0.0;

    // ---- s channel: A = Gamma(s, w1'-w, w-w2'), B = Gamma(s, w-w1, w-w2)
    // ---- u channel: A = Gamma(w1+w, w-w2', u),  B = Gamma(w1'+w, w2-w, u)
    for (int pass = 0; pass < 2; ++pass) {
        const int ch = pass == 0 ? 0 : 2;
        const int iv = pass == 0 ? ia : ic;
        const int cnt = A.tab_n[ch * nf + iv];
        const double* tw = A.tab_w + (long)(ch * nf + iv) * nq;
        const double* tg = A.tab_g + (long)(ch * nf + iv) * nq;
        for (int k = tid; k < cnt; k += kThreads) {
            const double om = tw[k];
            if (pass == 0) {
                make_plan(A.w, nf, ns, s, w1p - om, om - w2p, plan[k]);
                make_plan(A.w, nf, ns, s, om - w1, om - w2, plan[nq + k]);
            } else {
                make_plan(A.w, nf, ns, w1 + om, om - w2p, u, plan[k]);
                make_plan(A.w, nf, ns, w1p + om, w2 - om, u, plan[nq + k]);
            }
        }
        __syncthreads();
        if (act) {
            const double sgn = pass == 0 ? -2.0 : 2.0;
            for (int k = g; k < cnt; k += G) {
                double as, ad, bs, bd;
                eval_plan(plan[k], gs, gd, A.swap, p, as, ad);
                eval_plan(plan[nq + k], gs, gd, A.swap, p, bs, bd);
                const double W = tg[k];
                acc_s = fma(W, sgn * as * bs + as * bd + ad * bs, acc_s);
                acc_d = fma(W, 3.0 * as * bs + ad * bd, acc_d);
            }
        }
        __syncthreads();
    }

    // ---- t channel
    //   RPA:  -sum_j Gamma_{i1 j}(w1+w, t, w1'-w) Gamma_{j i2}(w+w2', t, w-w2)
    //   corr: Gamma_{i1i2}(w1+w, t, w1'-w) Gamma_{i2i2}(w2'+w, w2-w, -t)
    //       + Gamma_{i1i1}(w1+w, w-w1', -t) Gamma_{i1i2}(w+w2', t, w-w2)
    const int cnt = A.tab_n[1 * nf + it];
    const double* tw = A.tab_w + (long)(1 * nf + it) * nq;
    const double* tg = A.tab_g + (long)(1 * nf + it) * nq;
    for (int k = tid; k < cnt; k += kThreads) {
        const double om = tw[k];
        make_plan(A.w, nf, ns, w1 + om, t, w1p - om, plan[k]);
        make_plan(A.w, nf, ns, om + w2p, t, om - w2, plan[nq + k]);
        Plan P;
        make_plan(A.w, nf, ns, w2p + om, w2 - om, -t, P);
        eval_plan(P, gs, gd, A.swap, 0, onsite[4 * k + 0], onsite[4 * k + 1]);
        make_plan(A.w, nf, ns, w1 + om, om - w1p, -t, P);
        eval_plan(P, gs, gd, A.swap, 0, onsite[4 * k + 2], onsite[4 * k + 3]);
    }
    __syncthreads();

    // lattice-sum matrix entries owned by this thread (ns*ns <= 4*kThreads)
    double mss[4] = {0.0, 0.0, 0.0, 0.0}, mdd[4] = {0.0, 0.0, 0.0, 0.0};
    const int nm = ns * ns;
    for (int k0 = 0; k0 < cnt; k0 += kChunk) {
        const int kc = min(kChunk, cnt - k0);
        for (int i = tid; i < kc * ns; i += kThreads) {
            const int kk = i / ns, j = i % ns;
            double as, ad, bs, bd;
            eval_plan(plan[k0 + kk], gs, gd, A.swap, j, as, ad);
            eval_plan(plan[nq + k0 + kk], gs, gd, A.swap, j, bs, bd);
            vch[(0 * kChunk + kk) * ns + j] = as;
            vch[(1 * kChunk + kk) * ns + j] = ad;
            vch[(2 * kChunk + kk) * ns + j] = bs;
            vch[(3 * kChunk + kk) * ns + j] = bd;
        }
        __syncthreads();
        for (int e = tid, r = 0; e < nm; e += kThreads, ++r) {
            const int ka = e / ns, kb = e % ns;
            double ms = mss[r], md = mdd[r];
            for (int kk = 0; kk < kc; ++kk) {
                const double W = tg[k0 + kk];
                ms = fma(W * vch[(0 * kChunk + kk) * ns + ka], vch[(2 * kChunk + kk) * ns + kb], ms);
                md = fma(W * vch[(1 * kChunk + kk) * ns + ka], vch[(3 * kChunk + kk) * ns + kb], md);
            }
            mss[r] = ms; mdd[r] = md;
        }
        if (act) {
            for (int kk = g; kk < kc; kk += G) {
                const double as = vch[(0 * kChunk + kk) * ns + p], ad = vch[(1 * kChunk + kk) * ns + p];
                const double bs = vch[(2 * kChunk + kk) * ns + p], bd = vch[(3 * kChunk + kk) * ns + p];
                const double* o = onsite + 4 * (k0 + kk);
                const double o1s = o[0], o1d = o[1], o2s = o[2], o2d = o[3];
                const double W = tg[k0 + kk];
                acc_s = fma(W, -as * o1s + as * o1d - o2s * bs + o2d * bs, acc_s);
                acc_d = fma(W, 3.0 * ad * o1s + ad * o1d + 3.0 * o2s * bd + o2d * bd, acc_d);
            }
        }
        __syncthreads();
    }
    for (int e = tid, r = 0; e < nm; e += kThreads, ++r) {
        mat[e] = mss[r];
        mat[nm + e] = mdd[r];
    }

    // reduce the per-group partial sums over g
    red[tid] = act ? acc_s : 0.0;
    red[kThreads + tid] = act ? acc_d : 0.0;
    __syncthreads();
    if (tid < ns) {
        double ts = 0.0, td = 0.0;
        for (int gg = 0; gg < G; ++gg) {
            ts += red[gg * ns + tid];
            td += red[kThreads + gg * ns + tid];
        }
        double rs = 0.0, rd = 0.0;
        for (int q = A.rpa_off[tid]; q < A.rpa_off[tid + 1]; ++q) {
            const int e = A.rpa_ka[q] * ns + A.rpa_kb[q];
            const double cw = (double)A.rpa_cnt[q];
            rs = fma(cw, mat[e], rs);
            rd = fma(cw, mat[nm + e], rd);
        }
        const long o = (long)tau * ns + tid;
        dx[nf + o] = ts - 2.0 * rs;
        dx[nf + vsz + o] = td - 2.0 * rd;
    }
}

}  // namespace pffrg
