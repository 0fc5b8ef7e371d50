// kernels_xyz.h -- HIP kernels of the XYZ pf-FRG right-hand side (gfx950).
//
// XYZ models (arXiv:2109.13317, Sec. 2: H = sum Jx S^x S^x + Jy S^y S^y +
// Jz S^z S^z) keep only the diagonal vertex components (Sec. 3): three spin
// strains Gamma^{11}, Gamma^{22}, Gamma^{33} (x, y, z) and the density strain
// Gamma^{00} (d).  Every component obeys the symmetry relations of Eq. 18 as
// its SU(2) counterpart does (the spin strains are even under s <-> u, the
// density strain odd), so the node tables, interpolation plans and mesh
// look-ups of kernels_flow.h serve unchanged.  State: sig | Gx | Gy | Gz | Gd,
// each strain in the SU(2) strain layout.  The vertex is packed as (x, y, z, d)
// per element, 32 bytes: one interpolation corner is two 16-byte loads.
//
// Channel algebra (Eq. 24 contracted with Eq. 25, diagonal components; A, B
// the two vertices of each product in the paper's order; (a, b, c) cyclic in
// (x, y, z)):
//   s: dGd = Ad Bd + Ax Bx + Ay By + Az Bz,  dGa = Ad Ba + Aa Bd - Ab Bc - Ac Bb
//   u: dGd = Ad Bd + Ax Bx + Ay By + Az Bz,  dGa = Ad Ba + Aa Bd + Ab Bc + Ac Bb
//   t: dGm = -2 sum_j a_jm b_jm + Am sum_n e(m,n) O1n + Bm sum_n e(m,n) O2n,
//      e(m,n) = +1 if m or n is d or m = n, else -1 (O1, O2 the on-site vertices
//      of the two corrections);
// self-energy (Eq. 23): F = 2 sum_r mult_r Gd_r(w+x, 0, w-x) - (Gx+Gy+Gz+Gd)_0(w+x, x-w, 0);
// correlations (Eq. 30): chi^m direct 4 G^m_ij, on-site exchange -2 sum_n e(m,n) G^n_ii.
// With Gx = Gy = Gz these reduce to the SU(2) equations of kernels_flow.h.
#pragma once

#include "kernels_flow.h"
#include "kernels_obs.h"

namespace pffrg {

constexpr int kXyzMaxPairs = 16;     // one 16x16 matrix-core tile per strain in the t channel

// e(m, n) of the t-channel corrections and the correlations (m, n in x, y, z, d = 0..3).
__host__ __device__ constexpr double xyz_e(int m, int n) { return (m == 3 || n == 3 || m == n) ? 1.0 : -1.0; }

// One strain of pair p through a plan: the spin weights (x, y, z) or the
// density weights (d, which carry the s <-> u signs).
__device__ __forceinline__ double eval_strain(const Plan& P, const double* __restrict__ g,
                                              const int* __restrict__ swap, int p, bool density) {
    const int q = P.swp ? swap[p] : p;
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) a = fma(density ? P.wd[i] : P.ws[i], g[P.off[i] + q], a);
    return a;
}

// ------------------------------------------------------------ self-energy -

static __global__ void __launch_bounds__(kWave)
k_xyz_sigma(FlowArgs A, double lam, const double* __restrict__ x, long nv, double* __restrict__ dsig) {
    __shared__ MeshLds M;
    M.load(A, x, nullptr, threadIdx.x);
    A.w = M.w;
    const int n = blockIdx.x, lane = threadIdx.x;
    const double wn = A.w[n];
    const double* g = x + A.nf;          // strain m at g + m * nv
    // lanes 0..31 take x = +Lambda, lanes 32..63 x = -Lambda; lane r of a half
    // reads pair r, its lane 0 also the on-site exchange term
    const int half = lane >> 5, r = lane & 31;
    const double xx = half == 0 ? lam : -lam;
    Plan P;
    make_plan(A.w, A.nf, A.ns, wn + xx, 0.0, wn - xx, 1, 0, P);
    double f = 0.0;
    if (r < A.ns) f = 2.0 * (double)A.mult[r] * eval_strain(P, g + 3 * nv, A.swap, r, true);
    if (r == 0) {
        Plan Q;
        make_plan(A.w, A.nf, A.ns, wn + xx, xx - wn, 0.0, 2, 0, Q);
        double e = 0.0;
        for (int m = 0; m < 4; ++m) e += eval_strain(Q, g + m * nv, A.swap, 0, m == 3);
        f -= e;
    }
    for (int o = 16; o > 0; o >>= 1) f += __shfl_xor(f, o, kWave);
    const double term = f / (xx - odd_interp(A.w, A.nf, M.sig, xx));
    const double other = __shfl(term, 32, kWave);
    if (lane == 0) dsig[n] = (term + other) * kInvTwoPi;
}

// The four strains interleaved per element: gv[i] = (x, y, z, d), in the
// precision R of the vertex kernels (32 bytes per element in FP64, 16 in FP32).
template <class R>
static __global__ void k_xyz_pack(long n, const double* __restrict__ g, V4<R>* __restrict__ gv) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        V4<R> v;
        v.x = (R)g[i];
        v.y = (R)g[n + i];
        v.z = (R)g[2 * n + i];
        v.w = (R)g[3 * n + i];
        gv[i] = v;
    }
}

// Initial condition (Eq. 14, Eq. 21): sig = 0, G^m = J^m/4 for m = x, y, z
// (coupling3[m * ns + p]), Gd = 0.
static __global__ void k_xyz_init_state(long n, int nf, int ns, const double* __restrict__ coupling3,
                                        double* __restrict__ x) {
    const long vsz = (long)nf * (nf + 1) / 2 * nf * ns;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (i >= nf && i < nf + 3 * vsz) {
            const long j = i - nf;
            v = 0.25 * coupling3[(j / vsz) * ns + (j % vsz) % ns];
        }
        x[i] = v;
    }
}

// Bytes of one packed element (x, y, z, d).
template <class R> constexpr int kXyzElemBytes = 4 * (int)sizeof(R);

// One packed corner (x, y, z, d) at byte offset off: two 16-byte loads in
// FP64, one in FP32.
__device__ __forceinline__ void load_xyzd(__amdgpu_buffer_rsrc_t r, unsigned off, double (&v)[4]) {
    const double2 a = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
    const double2 b = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)(off + 16u), 0, 0));
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load_xyzd(__amdgpu_buffer_rsrc_t r, unsigned off, float (&v)[4]) {
    const float4 a = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// One interpolated vertex (four strains) of the pair at byte offsets pp
// (pp.y the exchanged pair) through plan P (offsets in bytes), in precision
// R: all corner loads are issued before the arithmetic.
template <class R>
__device__ __forceinline__ void eval_xyz(const PlanT<R>& P, __amdgpu_buffer_rsrc_t r, int2 pp, R (&v)[4]) {
    const unsigned q = P.swp ? pp.y : pp.x;
    R c[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) load_xyzd(r, (unsigned)P.off[i] + q, c[i]);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        R a = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) a = fmr(m == 3 ? P.wd[i] : P.ws[i], c[i][m], a);
        v[m] = a;
    }
}

template <class R>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t xyz_rsrc(const V4<R>* gv, long n) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)gv, (short)0, (int)(n * kXyzElemBytes<R>), 0x00020000);
}

// Plan offsets (elements) as byte offsets of the packed vertex.
template <class R>
__device__ __forceinline__ void to_bytes_xyz(PlanT<R>& P) {
#pragma unroll
    for (int i = 0; i < 4; ++i) P.off[i] *= kXyzElemBytes<R>;
}

// Sum the per-group partials acc[m] of lanes (g, p) over the groups and
// write (or add) the four strains of every pair; red: [4][64] doubles of LDS.
__device__ __forceinline__ void finish_xyz(double* red, int lane, int ns, int G, bool act, const double (&acc)[4],
                                           double* __restrict__ dx, long vsz, long out, bool add) {
#pragma unroll
    for (int m = 0; m < 4; ++m) red[m * kWave + lane] = act ? acc[m] : 0.0;
    wave_lds_sync();
    if (lane < ns) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double t = 0.0;
            for (int gg = 0; gg < G; ++gg) t += red[m * kWave + gg * ns + lane];
            double* d = dx + m * vsz + out * ns + lane;
            if (add) *d += t;
            else *d = t;
        }
    }
}

// Per-wave LDS of the XYZ kernels (bytes) in precision R: s/u plans
// [2][kPlanChunk], node weights (FP64), the reduction area; t plans
// [2][kTChunk], on-site values [2][4][kTChunk], weights, site vectors
// [8][4][16], the lattice-sum matrix (ns*ns, FP64) and the reduction area
// (the t layout is the larger one).
template <class R>
struct XyzWaveLds {
    static constexpr size_t su_plans() { return (size_t)2 * kPlanChunk * sizeof(PlanT<R>); }
    static constexpr size_t su_w() { return (size_t)kPlanChunk * sizeof(double); }
    static constexpr size_t t_plans() { return (size_t)2 * kTChunk * sizeof(PlanT<R>); }
    static constexpr size_t t_ons() { return (size_t)8 * kTChunk * sizeof(R); }
    static constexpr size_t t_w() { return (size_t)kTChunk * sizeof(R); }
    static constexpr size_t t_vb() { return (size_t)8 * 4 * 16 * sizeof(R); }
    static constexpr size_t mat() { return (size_t)kXyzMaxPairs * kXyzMaxPairs * sizeof(double); }
    static constexpr size_t red() { return (size_t)4 * kWave * sizeof(double); }
    static constexpr size_t su_bytes() { return su_plans() + su_w() + red(); }
    static constexpr size_t t_work() { return ((t_plans() + t_ons() + t_w() + t_vb()) + 15) & ~(size_t)15; }
    static constexpr size_t t_bytes() { return (t_work() > mat() ? t_work() : mat()) + red(); }
    static constexpr size_t bytes() { return ((su_bytes() > t_bytes() ? su_bytes() : t_bytes()) + 31) & ~(size_t)31; }
};

// ------------------------------------------------------------------ s, u -

// One wave per (s,t,u) triple, lanes (g, p): channel CH = 0 (s) or 2 (u);
// the s launch writes dGamma, the u launch adds.  R: precision of the
// interpolation and products; in FP32 the chunk sums are folded into
// compensated sums (CompSum), the results are FP64.
template <int CH, class R>
static __global__ void __launch_bounds__(kWave * kWavesPerBlock)
k_xyz_su(FlowArgs A, const V4<R>* __restrict__ gv, const int* __restrict__ uo_a, const int* __restrict__ uo_c,
         int n_triples, double* __restrict__ dx) {
    extern __shared__ __align__(32) unsigned char lds_raw[];
    using L = XyzWaveLds<R>;
    const int nf = A.nf, ns = A.ns, nq = A.nq;
    const Shared sh = load_shared(A, lds_raw, false);
    A.w = sh.w;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    unsigned char* base = lds_raw + SharedLds{nf, ns, A.n_terms}.bytes(false) + wid * L::bytes();
    PlanT<R>* plan = reinterpret_cast<PlanT<R>*>(base);
    double* wts = reinterpret_cast<double*>(base + L::su_plans());
    double* red = reinterpret_cast<double*>(base + L::su_plans() + L::su_w());
    const int o = xcd_order(n_triples);
    if (o < 0) return;
    const int q = o / nf, it = o % nf;
    const int ia = CH == 0 ? A.su_a[q] : uo_a[q];
    const int ic = CH == 0 ? A.su_c[q] : uo_c[q];
    const Triple T = make_triple(A.w, nf, ia, it, ic);
    const long vsz = (long)n_triples * ns;
    const __amdgpu_buffer_rsrc_t rv = xyz_rsrc<R>(gv, vsz);
    const int G = kWave / ns, g = lane / ns, p = lane % ns;
    const bool act = g < G;
    const int2 pp = make_int2(kXyzElemBytes<R> * p, kXyzElemBytes<R> * sh.swap[p]);
    const int iv = CH == 0 ? ia : ic;
    const int cnt = A.tab_n[CH * nf + iv];
    const double* tw = A.tab_w + (long)(CH * nf + iv) * nq;
    const double* tg = A.tab_g + (long)(CH * nf + iv) * nq;
    const R cross = CH == 0 ? R(-1) : R(1);
    R acc[4] = {0, 0, 0, 0};
    CompSum<R> sum[4];
    for (int k0 = 0; k0 < cnt; k0 += kPlanChunk) {
        const int kc = min(kPlanChunk, cnt - k0);
        {
            const int j = lane % kPlanChunk, vec = lane / kPlanChunk;
            if (j < kc) {
                const double om = tw[k0 + j];
                PlanT<R> P;
                if (CH == 0)
                    make_plan(A.w, nf, ns, T.s, vec == 0 ? T.w1p - om : om - T.w1, vec == 0 ? om - T.w2p : om - T.w2,
                              0, ia, P, &sh.lut);
                else
                    make_plan(A.w, nf, ns, vec == 0 ? T.w1 + om : T.w1p + om, vec == 0 ? om - T.w2p : T.w2 - om, T.u,
                              2, ic, P, &sh.lut);
                to_bytes_xyz(P);
                plan[vec * kPlanChunk + j] = P;
                if (vec == 0) wts[j] = tg[k0 + j];
            }
        }
        wave_lds_sync();
        if (act) {
            for (int k = g; k < kc; k += G) {
                R a[4], b[4];
                eval_xyz<R>(plan[k], rv, pp, a);
                eval_xyz<R>(plan[kPlanChunk + k], rv, pp, b);
                const R W = (R)wts[k];
                acc[3] = fmr(W, a[3] * b[3] + a[0] * b[0] + a[1] * b[1] + a[2] * b[2], acc[3]);
                acc[0] = fmr(W, a[3] * b[0] + a[0] * b[3] + cross * (a[1] * b[2] + a[2] * b[1]), acc[0]);
                acc[1] = fmr(W, a[3] * b[1] + a[1] * b[3] + cross * (a[2] * b[0] + a[0] * b[2]), acc[1]);
                acc[2] = fmr(W, a[3] * b[2] + a[2] * b[3] + cross * (a[0] * b[1] + a[1] * b[0]), acc[2]);
            }
        }
        if constexpr (sizeof(R) == 4) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                sum[m].add(acc[m]);
                acc[m] = R(0);
            }
        }
        wave_lds_sync();
    }
    double out[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if constexpr (sizeof(R) == 8) sum[m].s = acc[m];
        out[m] = sum[m].value();
    }
    finish_xyz(red, lane, ns, G, act, out, dx + nf, vsz, T.out, CH != 0);
}

// ---------------------------------------------------------------------- t -

// One wave per triple, ordered by (t, s, u); adds to dGamma.  The lattice
// sum of each strain m is the matrix M_m = sum_k W_k a_km b_km^T on one
// 16x16 matrix-core tile (four nodes per step, operands from the site
// vectors in LDS), contracted with the tabulated (ka, kb, count) terms.  In
// FP32 the tile and the vertex corrections of each plan chunk are folded
// into compensated sums; the contraction runs in FP64.
template <class R>
static __global__ void __launch_bounds__(kWave * kWavesPerBlock)
k_xyz_t(FlowArgs A, const V4<R>* __restrict__ gv, int n_triples, double* __restrict__ dx, int add) {
    constexpr bool kComp = sizeof(R) == 4;
    extern __shared__ __align__(32) unsigned char lds_raw[];
    using L = XyzWaveLds<R>;
    const int nf = A.nf, ns = A.ns, nq = A.nq;
    const Shared sh = load_shared(A, lds_raw, true);
    A.w = sh.w;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    unsigned char* base = lds_raw + SharedLds{nf, ns, A.n_terms}.bytes(true) + wid * L::bytes();
    PlanT<R>* plan = reinterpret_cast<PlanT<R>*>(base);                                    // [2][kTChunk]
    R* ons = reinterpret_cast<R*>(base + L::t_plans());                                    // [2][4][kTChunk]
    R* wts = reinterpret_cast<R*>(base + L::t_plans() + L::t_ons());                       // [kTChunk]
    R* vb = reinterpret_cast<R*>(base + L::t_plans() + L::t_ons() + L::t_w());             // [8][4][16]
    double* mat = reinterpret_cast<double*>(base);                                         // [ns*ns] at the end
    double* red = reinterpret_cast<double*>(base + L::t_bytes() - L::red());
    const int o = xcd_order(n_triples);
    if (o < 0) return;
    const int nsu = nf * (nf + 1) / 2;
    const int it = o / nsu, su = o % nsu;
    const Triple T = make_triple(A.w, nf, A.su_a[su], it, A.su_c[su]);
    const double t = T.t;
    const long vsz = (long)n_triples * ns;
    const __amdgpu_buffer_rsrc_t rv = xyz_rsrc<R>(gv, vsz);
    const int G = kWave / ns, g = lane / ns, p = lane % ns;
    const bool act = g < G;
    const int2 pp = make_int2(kXyzElemBytes<R> * p, kXyzElemBytes<R> * sh.swap[p]);
    const int cnt = A.tab_n[1 * nf + it];
    const double* tw = A.tab_w + (long)(1 * nf + it) * nq;
    const double* tg = A.tab_g + (long)(1 * nf + it) * nq;
    R acc[4] = {0, 0, 0, 0};                         // vertex corrections of pair p (lanes (g, p))
    CompSum<R> sacc[4];
    Vec4<R> cm[4];
    CompSum<R> ccm[kComp ? 4 : 1][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) cm[m] = Vec4<R>{0, 0, 0, 0};
    for (int i = lane; i < 8 * 4 * 16; i += kWave) vb[i] = R(0);     // padding pairs stay zero
    for (int k0 = 0; k0 < cnt; k0 += kTChunk) {
        const int kc = min(kTChunk, cnt - k0);
        {
            // lane (role, j): role 0/1 the site-vector plans a/b of node j,
            // role 2/3 the on-site vertices (pair 0, all strains) of the corrections
            const int j = lane % kTChunk, role = lane / kTChunk;
            if (j < kc) {
                const double om = tw[k0 + j];
                const double a0 = role == 0 ? T.w1 + om : (role == 1 ? om + T.w2p : (role == 2 ? T.w2p + om : T.w1 + om));
                const double a1 = role == 0 ? t : (role == 1 ? t : (role == 2 ? T.w2 - om : om - T.w1p));
                const double a2 = role == 0 ? T.w1p - om : (role == 1 ? om - T.w2 : -t);
                PlanT<R> P;
                make_plan(A.w, nf, ns, a0, a1, a2, role < 2 ? 1 : 2, it, P, &sh.lut);
                to_bytes_xyz(P);
                if (role < 2) {
                    plan[role * kTChunk + j] = P;
                    if (role == 0) wts[j] = (R)tg[k0 + j];
                } else {
                    R v[4];
                    eval_xyz<R>(P, rv, make_int2(0, kXyzElemBytes<R> * sh.swap[0]), v);
#pragma unroll
                    for (int m = 0; m < 4; ++m) ons[((role - 2) * 4 + m) * kTChunk + j] = v[m];
                }
            }
        }
        wave_lds_sync();
        for (int s0 = 0; s0 < kc; s0 += 4) {
            const int sc = min(4, kc - s0);
            if (act && g < sc) {
                const int k = s0 + g;
                R a[4], b[4];
                eval_xyz<R>(plan[k], rv, pp, a);
                eval_xyz<R>(plan[kTChunk + k], rv, pp, b);
                const R W = wts[k];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    vb[(m * 4 + g) * 16 + p] = W * a[m];
                    vb[((4 + m) * 4 + g) * 16 + p] = b[m];
                    R c1 = 0, c2 = 0;
#pragma unroll
                    for (int n = 0; n < 4; ++n) {
                        c1 = fmr((R)xyz_e(m, n), ons[(0 * 4 + n) * kTChunk + k], c1);
                        c2 = fmr((R)xyz_e(m, n), ons[(1 * 4 + n) * kTChunk + k], c2);
                    }
                    acc[m] = fmr(W, a[m] * c1 + b[m] * c2, acc[m]);
                }
            }
            wave_lds_sync();
            {
                const int i16 = lane % 16, k4 = lane / 16;
                const bool in = k4 < sc;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const R xa = in ? vb[(m * 4 + k4) * 16 + i16] : R(0);
                    const R xb = in ? vb[((4 + m) * 4 + k4) * 16 + i16] : R(0);
                    cm[m] = mfma16x16x4<R>(xa, xb, cm[m]);
                }
            }
            wave_lds_sync();
            // the site vectors of the next sub-chunk overwrite these rows; rows of
            // nodes it does not fill are masked by `in` above
        }
        if constexpr (kComp) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                sacc[m].add(acc[m]);
                acc[m] = R(0);
#pragma unroll
                for (int r = 0; r < 4; ++r) ccm[m][r].add(cm[m][r]);
                cm[m] = Vec4<R>{0, 0, 0, 0};
            }
        }
    }
    // contract each strain's matrix with the tabulated terms
    wave_lds_sync();
    double tot[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ka = mfma_row<R>(lane, r), kb = lane % 16;
            double v;
            if constexpr (kComp) v = ccm[m][r].value();
            else v = (double)cm[m][r];
            if (ka < ns && kb < ns) mat[ka * ns + kb] = v;
        }
        wave_lds_sync();
        double sv = 0.0;
        if (act)
            for (int qq = sh.off[p] + g; qq < sh.off[p + 1]; qq += G) {
                const int tq = sh.terms[qq];
                sv = fma((double)(tq >> 16), mat[tq & 0xffff], sv);
            }
        double av;
        if constexpr (kComp) av = sacc[m].value();
        else av = (double)acc[m];
        tot[m] = fma(-2.0, sv, act ? av : 0.0);
        wave_lds_sync();
    }
    finish_xyz(red, lane, ns, G, act, tot, dx + nf, vsz, T.out, add != 0);
}

// t channel, four waves per triple (one workgroup): wave h holds the
// lattice-sum matrix of strain h only, NT x NT tiles (NT = 2 from 17 to 32
// pairs, where the four strains' tiles would need 128 accumulation registers
// in one wave; NT = 1 up to 16 pairs).  The nodes go in sub-chunks of 4 NG
// (NG = 64 / (16 NT) node groups of lanes per wave): wave h gathers nodes
// NG h .. NG h + NG - 1 (both vectors, all four strains, and their vertex
// corrections) into the triple's site-vector buffer, then every wave adds the
// sub-chunk to its strain's matrix (NG matrix-core steps).  Plans for 32
// nodes are built at once, one role per wave (site vectors a and b, the two
// on-site vertices).  At the end wave m writes its matrix and the lanes of
// all four waves contract it with the tabulated terms, strain by strain;
// wave m adds strain m of every pair to dGamma.  In FP32 the matrix tiles and
// the vertex corrections of each plan chunk are folded into compensated sums.
constexpr int kXyzMaxPairs4 = 32;
constexpr int kXyzT4Chunk = 32;

template <class R>
struct XyzT4Lds {
    static constexpr size_t plans() { return (size_t)2 * kXyzT4Chunk * sizeof(PlanT<R>); }
    static constexpr size_t ons() { return (size_t)(8 + 1) * kXyzT4Chunk * sizeof(R); }
    // 8 rows x (4 NG nodes) x (16 NT pairs) = 2048 values for either NT
    static constexpr size_t vb() { return (size_t)8 * 8 * kXyzMaxPairs4 * sizeof(R); }
    static constexpr size_t mat() { return (size_t)kXyzMaxPairs4 * kXyzMaxPairs4 * sizeof(double); }
    static constexpr size_t red() { return (size_t)16 * kWave * sizeof(double); }
    static constexpr size_t work() { return plans() + ons() + vb(); }
    static constexpr size_t area() { return ((work() > mat() ? work() : mat()) + 31) & ~(size_t)31; }
    // the partial sums reuse the area once the last contraction is done
    static constexpr size_t bytes() { return area() > red() ? area() : red(); }
};

template <int NT, class R>
static __global__ void __launch_bounds__(kWave * kWavesPerBlock)
__attribute__((amdgpu_waves_per_eu(4)))
k_xyz_t4(FlowArgs A, const V4<R>* __restrict__ gv, int n_triples, double* __restrict__ dx, int add) {
    constexpr int NG = 4 / NT;             // node groups of lanes per wave
    constexpr int SC = 4 * NG;             // nodes per sub-chunk
    constexpr int SP = 16 * NT;            // site-vector row stride (pairs)
    constexpr bool kComp = sizeof(R) == 4;
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int nf = A.nf, ns = A.ns, nq = A.nq;
    const Shared sh = load_shared(A, lds_raw, true);
    A.w = sh.w;
    using L = XyzT4Lds<R>;
    unsigned char* base = lds_raw + SharedLds{nf, ns, A.n_terms}.bytes(true);
    PlanT<R>* plan = reinterpret_cast<PlanT<R>*>(base);                          // [2][chunk]
    R* ons = reinterpret_cast<R*>(base + L::plans());                            // [2][4][chunk]
    R* wts = ons + 8 * kXyzT4Chunk;                                              // [chunk]
    R* vb = reinterpret_cast<R*>(base + L::plans() + L::ons());                  // [8 rows][SC nodes][SP]
    double* mat = reinterpret_cast<double*>(base);                               // [ns*ns] after the node loop
    double* red = reinterpret_cast<double*>(base);                               // [4 waves][4 strains][64] at the end
    const int h = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    // one triple per workgroup, each XCD a contiguous range in (t, s, u) order
    const int per = gridDim.x / 8;
    const int o = __builtin_amdgcn_readfirstlane((int)((blockIdx.x % 8) * per + blockIdx.x / 8));
    if (o >= n_triples) return;                  // the whole workgroup: no barrier is left behind
    const int nsu = nf * (nf + 1) / 2;
    const int it = o / nsu, su = o % nsu;
    const Triple T = make_triple(A.w, nf, A.su_a[su], it, A.su_c[su]);
    const double t = T.t;
    const long vsz = (long)n_triples * ns;
    const __amdgpu_buffer_rsrc_t rv = xyz_rsrc<R>(gv, vsz);
    const int g = lane / ns, p = lane % ns;      // node lanes: g < NG
    const int2 pp = make_int2(kXyzElemBytes<R> * p, kXyzElemBytes<R> * sh.swap[p]);
    const int cnt = A.tab_n[1 * nf + it];
    const double* tw = A.tab_w + (long)(1 * nf + it) * nq;
    const double* tg = A.tab_g + (long)(1 * nf + it) * nq;
    R acc[4] = {0, 0, 0, 0};                     // vertex corrections over this lane's nodes
    CompSum<R> sacc[4];
    Vec4<R> c[NT][NT];
    CompSum<R> cc[kComp ? NT : 1][kComp ? NT : 1][4];
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = 0; J < NT; ++J) c[I][J] = Vec4<R>{0, 0, 0, 0};
    for (int k0 = 0; k0 < cnt; k0 += kXyzT4Chunk) {
        const int kc = min(kXyzT4Chunk, cnt - k0);
        {
            // wave h builds the plans of role h for node j: 0/1 the site
            // vectors a/b, 2/3 the on-site vertices (pair 0, all strains)
            const int j = lane, role = h;
            if (j < kc) {
                const double om = tw[k0 + j];
                const double a0 = role == 0 ? T.w1 + om : (role == 1 ? om + T.w2p : (role == 2 ? T.w2p + om : T.w1 + om));
                const double a1 = role == 0 ? t : (role == 1 ? t : (role == 2 ? T.w2 - om : om - T.w1p));
                const double a2 = role == 0 ? T.w1p - om : (role == 1 ? om - T.w2 : -t);
                PlanT<R> P;
                make_plan(A.w, nf, ns, a0, a1, a2, role < 2 ? 1 : 2, it, P, &sh.lut);
                to_bytes_xyz(P);
                if (role < 2) {
                    plan[role * kXyzT4Chunk + j] = P;
                    if (role == 0) wts[j] = (R)tg[k0 + j];
                } else {
                    R v[4];
                    eval_xyz<R>(P, rv, make_int2(0, kXyzElemBytes<R> * sh.swap[0]), v);
#pragma unroll
                    for (int m = 0; m < 4; ++m) ons[((role - 2) * 4 + m) * kXyzT4Chunk + j] = v[m];
                }
            }
        }
        __syncthreads();
        for (int s0 = 0; s0 < kc; s0 += SC) {
            const int sc = min(SC, kc - s0);
            const int kk = NG * h + g;
            if (g < NG && kk < sc) {
                const int k = s0 + kk;
                R a[4], b[4];
                eval_xyz<R>(plan[k], rv, pp, a);
                eval_xyz<R>(plan[kXyzT4Chunk + k], rv, pp, b);
                const R W = wts[k];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    vb[(m * SC + kk) * SP + p] = W * a[m];
                    vb[((4 + m) * SC + kk) * SP + p] = b[m];
                    R c1 = 0, c2 = 0;
#pragma unroll
                    for (int n = 0; n < 4; ++n) {
                        c1 = fmr((R)xyz_e(m, n), ons[(0 * 4 + n) * kXyzT4Chunk + k], c1);
                        c2 = fmr((R)xyz_e(m, n), ons[(1 * 4 + n) * kXyzT4Chunk + k], c2);
                    }
                    acc[m] = fmr(W, a[m] * c1 + b[m] * c2, acc[m]);
                }
            }
            __syncthreads();
            // M_h[ka][kb] += (W a_h)[ka] b_h[kb] over the sub-chunk's nodes
            {
                const int i16 = lane % 16, k4 = lane / 16;
#pragma unroll
                for (int q = 0; q < NG; ++q) {
                    const int node = 4 * q + k4;
                    R xa[NT], xb[NT];
#pragma unroll
                    for (int I = 0; I < NT; ++I) {
                        const int pr = 16 * I + i16;
                        const bool in = node < sc && pr < ns;
                        const int off = in ? node * SP + pr : 0;
                        xa[I] = in ? vb[h * SC * SP + off] : R(0);
                        xb[I] = in ? vb[(4 + h) * SC * SP + off] : R(0);
                    }
#pragma unroll
                    for (int I = 0; I < NT; ++I)
#pragma unroll
                        for (int J = 0; J < NT; ++J) c[I][J] = mfma16x16x4<R>(xa[I], xb[J], c[I][J]);
                }
            }
            __syncthreads();
        }
        if constexpr (kComp) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                sacc[m].add(acc[m]);
                acc[m] = R(0);
            }
#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int J = 0; J < NT; ++J) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) cc[I][J][r].add(c[I][J][r]);
                    c[I][J] = Vec4<R>{0, 0, 0, 0};
                }
        }
    }
    // contraction with the tabulated terms, strain by strain: wave m writes
    // its matrix, the lanes (h, g < NG) of all waves take every (4 NG)-th term
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if (h == m) {
#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int J = 0; J < NT; ++J)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int ka = 16 * I + mfma_row<R>(lane, r), kb = 16 * J + lane % 16;
                        double v;
                        if constexpr (kComp) v = cc[I][J][r].value();
                        else v = (double)c[I][J][r];
                        if (ka < ns && kb < ns) mat[ka * ns + kb] = v;
                    }
        }
        __syncthreads();
        if (g < NG) {
            double sv = 0.0;
            for (int qq = sh.off[p] + NG * h + g; qq < sh.off[p + 1]; qq += 4 * NG) {
                const int tq = sh.terms[qq];
                sv = fma((double)(tq >> 16), mat[tq & 0xffff], sv);
            }
            tot[m] = sv;
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double av;
        if constexpr (kComp) av = sacc[m].value();
        else av = (double)acc[m];
        red[(h * 4 + m) * kWave + lane] = g < NG ? fma(-2.0, tot[m], av) : 0.0;
    }
    __syncthreads();
    // wave m adds strain m of every pair
    if (lane < ns) {
        const int m = h;
        double v = 0.0;
#pragma unroll
        for (int hh = 0; hh < 4; ++hh)
#pragma unroll
            for (int gg = 0; gg < NG; ++gg) v += red[(hh * 4 + m) * kWave + gg * ns + lane];
        double* d = dx + nf + m * vsz + T.out * ns + lane;
        if (add) *d += v;
        else *d = v;
    }
}

// ---------------------------------------------------------- correlations -

// Workgroup (p, slice): the part of the double integrals of pair p over the
// node pairs of its slice, per strain m: part[((p * slices + slice) * 4 + m].
static __global__ void __launch_bounds__(kChiThreads)
k_xyz_chi_pairs(const double* __restrict__ w, int nf, int ns, const int* __restrict__ swap,
                const double* __restrict__ x, const double* __restrict__ cw, const double* __restrict__ cq,
                const double* __restrict__ cg2, const int* __restrict__ cn, double* __restrict__ part) {
    __shared__ double rr[4][kChiThreads];
    const int p = blockIdx.x, sl = blockIdx.y, tid = threadIdx.x;
    const int n = *cn;
    const long vsz = (long)nf * (nf + 1) / 2 * nf * ns;
    const double* g = x + nf;
    const int nn = n * n;
    const int e0 = (int)((long)nn * sl / kChiSlices), e1 = (int)((long)nn * (sl + 1) / kChiSlices);
    double az[4] = {0.0, 0.0, 0.0, 0.0};
    for (int e = e0 + tid; e < e1; e += kChiThreads) {
        const int i = e / n, j = e % n;
        const double w1 = cw[i], w2 = cw[j];
        const double f = cq[i] * cq[j] * cg2[i] * cg2[j];
        Plan P;
        make_plan(w, nf, ns, w1 + w2, 0.0, w1 - w2, 1, 0, P);
        double tz[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) tz[m] = 4.0 * eval_strain(P, g + m * vsz, swap, p, m == 3);
        if (p == 0) {
            make_plan(w, nf, ns, w1 + w2, w2 - w1, 0.0, 2, 0, P);
            double ex[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) ex[m] = eval_strain(P, g + m * vsz, swap, 0, m == 3);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                double xm = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) xm = fma(xyz_e(m, q), ex[q], xm);
                tz[m] = fma(-2.0, xm, tz[m]);
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) az[m] = fma(f, tz[m], az[m]);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) rr[m][tid] = az[m];
    __syncthreads();
    for (int st = kChiThreads / 2; st > 0; st >>= 1) {
        if (tid < st)
#pragma unroll
            for (int m = 0; m < 4; ++m) rr[m][tid] += rr[m][tid + st];
        __syncthreads();
    }
    if (tid < 4) part[((long)p * kChiSlices + sl) * 4 + tid] = rr[tid][0];
}

// chi[m * ns + p] (m = x, y, z, d) from the slices, with the on-site one-loop term.
static __global__ void k_xyz_chi_final(int ns, const double* __restrict__ cq, const double* __restrict__ cg2,
                                       const int* __restrict__ cn, const double* __restrict__ part,
                                       double* __restrict__ chi) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ns) return;
    const double pref = 1.0 / (16.0 * M_PI * M_PI);
    double b = 0.0;
    if (p == 0) {
        for (int i = 0; i < *cn; ++i) b = fma(cq[i], cg2[i], b);
        b *= 0.5 * kInvTwoPi;        // 1/(4 pi)
    }
    for (int m = 0; m < 4; ++m) {
        double s = 0.0;
        for (int sl = 0; sl < kChiSlices; ++sl) s += part[((long)p * kChiSlices + sl) * 4 + m];
        chi[m * ns + p] = -pref * s + b;
    }
}

}  // namespace pffrg
