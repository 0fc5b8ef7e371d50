// kernels_tri.h -- HIP kernels of the general (TRI) pf-FRG right-hand side (gfx950).
//
// General time-reversal invariant models (arXiv:2109.13317, Sec. 2:
// H = sum J_ij^{mu nu} S_i^mu S_j^nu with real 3x3 matrices) keep all sixteen
// vertex components Gamma^{mu nu} (Sec. 3, Eq. 16), component index
// q = 4 mu + nu (0 the density index, 1..3 x, y, z).  Gamma^{mu nu} is real
// where xi(mu) xi(nu) = 1 and imaginary where it is -1 (Eq. 18); the state
// holds the real number r with Gamma = r, resp. Gamma = i r, sixteen strains
// of the SU(2) strain layout: sig | G^{00} | G^{01} | ... | G^{33}.
//
// Symmetries (Eq. 18) on top of the SU(2) ones: s -> -s and u -> -u transpose
// (mu <-> nu) besides exchanging the sites, t -> -t and u -> -u multiply by
// xi(mu) xi(nu), s <-> u by -xi(nu).  A plan of kernels_flow.h therefore
// serves once two flags are added: bit 0 of swp (exchanged sites) is also
// the transposition, bit 1 the xi xi sign; the s <-> u signs sit in the
// weights as for SU(2) (density weights for the stored nu = 0 components).
// The packed vertex holds, per frequency point, the sixteen components as
// eight 16-byte chunks, chunk-major: [point][chunk][pair], so that the eight
// loads of a corner are each one contiguous wave access over the pairs.
//
// Channel products.  In two-spin operator form (V = sum Gamma^{mu nu}
// sigma^mu (x) sigma^nu, Eq. 25) the spin sums of Eq. 24 give
//   s:  A B                                 sigma^m1 sigma^m2 (x) sigma^n1 sigma^n2
//   u:  the first spin's product reversed   sigma^m2 sigma^m1 (x) sigma^n1 sigma^n2
//   t:  RPA -sum_j: a trace over the inner legs, -2 Gamma_A^{m k} Gamma_B^{k n};
//       corrections (A, O1): sigma^m1 (x) sigma^m2 sigma^n1 sigma^n2,
//                   (O2, B): sigma^n1 sigma^m2 sigma^m1 (x) sigma^n2
// for components (m1 n1) of the first and (m2 n2) of the second vertex.  Every
// pair of input components feeds exactly one output component; with the i's
// of the real representation the coefficient is +-1 (+-2 for the RPA term).
// The tables are generated at compile time from the Pauli products
// sigma^a sigma^b = delta_ab + i eps_abc sigma^c.
// Self-energy (Eq. 23, the spin average, which keeps Sigma imaginary):
//   F = 2 sum_r mult_r G^{00}_r(w+x, 0, w-x) - (G^{00} + G^{11} + G^{22} + G^{33})_0(w+x, x-w, 0).
// Correlations (Eq. 30, real parts): chi^{mu nu} direct 4 Gamma^{mu nu}_ij,
// on-site exchange -tr(sigma^mu sigma^nu' sigma^nu sigma^mu') Gamma^{mu' nu'}_ii.
#pragma once

#include <utility>

#include "kernels_flow.h"
#include "kernels_obs.h"
#include "kernels_xyz.h"   // eval_strain

namespace pffrg {

constexpr int kTriComps = 16;
constexpr int kTriElemBytes = kTriComps * 8;      // one packed FP64 element
constexpr int kTriMaxPairs = 64;                  // one lane per pair at least
constexpr int kTriWaves = 2;                      // waves per workgroup of the vertex kernels

// ------------------------------------------------------- Pauli algebra -

struct PauliMul {
    int c, ph;      // sigma^a sigma^b = i^ph sigma^c
};

__host__ __device__ constexpr PauliMul pauli_mul(int a, int b) {
    return a == 0 ? PauliMul{b, 0}
         : b == 0 ? PauliMul{a, 0}
         : a == b ? PauliMul{0, 0}
                  : PauliMul{6 - a - b, (a % 3) + 1 == b ? 1 : 3};
}

// Power of i of component q in the real representation (1 where xi xi = -1).
__host__ __device__ constexpr int tri_ie(int q) { return ((q / 4 == 0) != (q % 4 == 0)) ? 1 : 0; }

// The transposed component index.
__host__ __device__ constexpr int tri_tr(int q) { return (q % 4) * 4 + q / 4; }

enum TriChannel { kTriS = 0, kTriU = 1, kTriC1 = 2, kTriC2 = 3, kTriRpa = 4 };

struct TriTerm {
    int c1, c2, q, k;   // acc[q] += k * A[c1] * B[c2]; k = 0: no term
};

__host__ __device__ constexpr TriTerm tri_term(int ch, int i) {
    const int c1 = i / 16, c2 = i % 16;
    const int m1 = c1 / 4, n1 = c1 % 4, m2 = c2 / 4, n2 = c2 % 4;
    int mu = 0, nu = 0, ph = 0, mult = 1;
    if (ch == kTriS) {
        const PauliMul a = pauli_mul(m1, m2), b = pauli_mul(n1, n2);
        mu = a.c; nu = b.c; ph = a.ph + b.ph;
    } else if (ch == kTriU) {
        const PauliMul a = pauli_mul(m2, m1), b = pauli_mul(n1, n2);
        mu = a.c; nu = b.c; ph = a.ph + b.ph;
    } else if (ch == kTriC1) {
        const PauliMul x = pauli_mul(m2, n1), y = pauli_mul(x.c, n2);
        mu = m1; nu = y.c; ph = x.ph + y.ph;
    } else if (ch == kTriC2) {
        const PauliMul x = pauli_mul(n1, m2), y = pauli_mul(x.c, m1);
        mu = y.c; nu = n2; ph = x.ph + y.ph;
    } else {
        if (n1 != m2) return TriTerm{c1, c2, 0, 0};
        mu = m1; nu = n2; ph = 2; mult = 2;       // -2 Gamma_A^{m1 k} Gamma_B^{k n2}
    }
    const int q = 4 * mu + nu;
    const int e = (ph + tri_ie(c1) + tri_ie(c2) - tri_ie(q) + 8) % 4;
    return TriTerm{c1, c2, q, e == 0 ? mult : (e == 2 ? -mult : 0)};
}

// Every term is real in the real representation (Eq. 18 closes the algebra).
__host__ __device__ constexpr bool tri_tables_real() {
    for (int ch = 0; ch <= kTriRpa; ++ch)
        for (int i = 0; i < 256; ++i) {
            const int c1 = i / 16, c2 = i % 16;
            if (ch == kTriRpa && c1 % 4 != c2 / 4) continue;
            if (tri_term(ch, i).k == 0) return false;
        }
    return true;
}
static_assert(tri_tables_real(), "TRI channel algebra must be real in the real representation");

template <int CH, int I>
__device__ __forceinline__ void tri_fma_one(const double (&a)[16], const double (&b)[16], double (&acc)[16]) {
    constexpr TriTerm T = tri_term(CH, I);
    if constexpr (T.k == 1) acc[T.q] = fma(a[T.c1], b[T.c2], acc[T.q]);
    else if constexpr (T.k == -1) acc[T.q] = fma(-a[T.c1], b[T.c2], acc[T.q]);
    else if constexpr (T.k != 0) acc[T.q] = fma((double)T.k * a[T.c1], b[T.c2], acc[T.q]);
}

template <int CH, int... I>
__device__ __forceinline__ void tri_product(const double (&a)[16], const double (&b)[16], double (&acc)[16],
                                            std::integer_sequence<int, I...>) {
    (tri_fma_one<CH, I>(a, b, acc), ...);
}

// acc += (A, B) through channel CH (fully unrolled, constant register indices).
template <int CH>
__device__ __forceinline__ void tri_mul(const double (&a)[16], const double (&b)[16], double (&acc)[16]) {
    tri_product<CH>(a, b, acc, std::make_integer_sequence<int, 256>{});
}

// Exchange coefficient of the correlations: X(m, q') = Re[i^{ie(q')} tr(sigma^mu sigma^nu'
// sigma^nu sigma^mu')] for m = 4 mu + nu, q' = 4 mu' + nu'.
__host__ __device__ constexpr int tri_chi_x(int m, int qp) {
    const int mu = m / 4, nu = m % 4, mp = qp / 4, np = qp % 4;
    const PauliMul a = pauli_mul(mu, np), b = pauli_mul(a.c, nu), c = pauli_mul(b.c, mp);
    if (c.c != 0) return 0;
    const int e = (a.ph + b.ph + c.ph + tri_ie(qp)) % 4;
    return e == 0 ? 2 : (e == 2 ? -2 : 0);
}

// ------------------------------------------------------ spin rotations -

// Lattice symmetries combined with a global spin transformation W (Sec. 4.1;
// W a signed permutation with det +1): Gamma_{i1 i2} = W Gamma_q W^T on the
// spin indices, so component m = 4 mu + nu of the mapped pair is
// s(mu) s(nu) Gamma_q^{pi(mu) pi(nu)}.  A rotation is tabulated as 16 words
// rot16[m] = (4 pi(mu) + pi(nu)) | (sign < 0) << 4.
__device__ __forceinline__ double tri_rot_get(const double* __restrict__ v, int word) {
    const double x = v[word & 15];
    return (word & 16) ? -x : x;
}

// Double index of component m of element (point, pair q) in the packed
// layout [point][chunk][pair] (chunk = two components).
__host__ __device__ __forceinline__ long tri_packed_index(long point, int q, int m, int ns) {
    return 2 * ((point * 8 + m / 2) * (long)ns + q) + (m & 1);
}

// The pre-rotated copy of the exchanged pairs: element (point, p) of the
// second half of gv is W Gamma W^T of element (point, swap[p]) of the first
// half, W = rotation swap_rot[p] (one thread per element).
static __global__ void k_tri_pack_swap(long n, int ns, const int* __restrict__ swap, const int* __restrict__ swap_rot,
                                       const int* __restrict__ rot16, double* __restrict__ gv) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int p = (int)(i % ns);
        const long pt = i / ns;
        const int* rw = rot16 + 16 * swap_rot[p];
        double* dst = gv + 16 * n;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int word = rw[m];
            const double x = gv[tri_packed_index(pt, swap[p], word & 15, ns)];
            dst[tri_packed_index(pt, p, m, ns)] = (word & 16) ? -x : x;
        }
    }
}

// chi of every (basis site, site) in the observable layout with the site's
// rotation: out[m * nbs + k] = (W chi_q W^T)^m, NaN past the range.
static __global__ void k_tri_chi_sites(int ns, int nbs, const int* __restrict__ site_pair,
                                       const int* __restrict__ site_rot, const int* __restrict__ rot16,
                                       const double* __restrict__ chi, double* __restrict__ out) {
    const long n = 16L * nbs;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int m = (int)(i / nbs), k = (int)(i % nbs);
        const int sp = site_pair[k];
        if (sp < 0) {
            out[i] = __builtin_nan("");
            continue;
        }
        const int word = rot16[16 * site_rot[k] + m];
        const double x = chi[(word & 15) * ns + sp];
        out[i] = (word & 16) ? -x : x;
    }
}

// Terms of the lattice sum with rotations: word ra | rb << 8 per term.
struct TriRotLds {
    int n_terms, n_rot;
    __host__ __device__ size_t bytes() const {
        return n_rot > 1 ? (((size_t)(n_terms + 16 * n_rot) * sizeof(int)) + 31) & ~(size_t)31 : 0;
    }
};

// ------------------------------------------------------------- plans -

// Flags of a TRI plan on top of make_plan's: bit 1 = the xi xi sign (an odd
// number of the t -> -t and u -> -u relations); bit 0 (make_plan's swp) is
// the site exchange and the transposition.
__device__ __forceinline__ void make_plan_tri(const double* __restrict__ w, int nf, int ns, double s, double t,
                                              double u, int kslot, int kidx, Plan& P, const MeshLut* lut) {
    make_plan(w, nf, ns, s, t, u, kslot, kidx, P, lut);
    P.swp |= (int)((t < 0.0) != (u < 0.0)) << 1;
}

// Apply a plan's transposition and sign to the sixteen interpolated stored
// components.  Every index is a template argument: written as a loop over
// m, c[tri_tr(m)] was lowered as a run-time index into the register array
// (a compare and select for each of the sixteen elements, per component);
// the sign is an xor of the high word.
template <int M>
__device__ __forceinline__ void tri_finish_one(bool tr, unsigned sg, const double (&c)[16], double (&v)[16]) {
    constexpr int T = tri_tr(M);
    const double val = tr ? c[T] : c[M];
    if constexpr (tri_ie(M) != 0)
        v[M] = __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, val) ^ ((unsigned long long)sg << 32));
    else
        v[M] = val;
}
template <int... M>
__device__ __forceinline__ void tri_finish_all(bool tr, unsigned sg, const double (&c)[16], double (&v)[16],
                                               std::integer_sequence<int, M...>) {
    (tri_finish_one<M>(tr, sg, c, v), ...);
}
__device__ __forceinline__ void tri_finish(int flags, const double (&c)[16], double (&v)[16]) {
    tri_finish_all((flags & 1) != 0, (flags & 2) ? 0x80000000u : 0u, c, v, std::make_integer_sequence<int, 16>{});
}

// Sixteen components of pair p from the strain-major state g (strain q at
// g + q * vsz) through a TRI plan (element offsets).  swap_words: the
// rotation words of the exchanged pair (spin permutations; NULL: none), read
// as permuted strain addresses.
__device__ __forceinline__ void eval_tri_state(const Plan& P, const double* __restrict__ g, long vsz,
                                               const int* __restrict__ swap, int p, double (&v)[16],
                                               const int* __restrict__ swap_words = nullptr) {
    const bool sw = P.swp & 1;
    const int qp = sw ? swap[p] : p;
    double c[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int word = (sw && swap_words) ? swap_words[m] : m;
        const double* gs = g + (word & 15) * vsz;
        double a = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) a = fma(m % 4 == 0 ? P.wd[i] : P.ws[i], gs[P.off[i] + qp], a);
        c[m] = (word & 16) ? -a : a;
    }
    tri_finish(P.swp, c, v);
}

// The size is made wave-uniform explicitly: computed from a select on the
// kernel argument swap_copy it could land in vector registers, and a
// descriptor there costs a readfirstlane loop around every load.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tri_rsrc(const double* gv, long n) {
    const int bytes = __builtin_amdgcn_readfirstlane((int)(n * kTriElemBytes));
    return __builtin_amdgcn_make_buffer_rsrc((void*)gv, (short)0, bytes, 0x00020000);
}

// Plan offsets (elements, point * ns) as byte offsets of the packed vertex:
// a point's block is ns * 128 bytes.
__device__ __forceinline__ void to_bytes_tri(Plan& P) {
#pragma unroll
    for (int i = 0; i < 4; ++i) P.off[i] *= kTriElemBytes;
}

// Sixteen components of the pair at byte offsets pp (16 * pair within a
// chunk row; pp.y the exchanged pair) through a plan with byte offsets,
// chunk rows hstride = 16 * ns bytes apart: corner by corner, eight 16-byte
// loads each, the corner's loads issued before its arithmetic.
__device__ __forceinline__ void eval_tri(const Plan& P, __amdgpu_buffer_rsrc_t r, int2 pp, unsigned hstride,
                                         double (&v)[16]) {
    const unsigned q = (P.swp & 1) ? pp.y : pp.x;
    double c[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) c[m] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double e[16];
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const double2 d = __builtin_bit_cast(
                double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)((unsigned)P.off[i] + q + hstride * h), 0, 0));
            e[2 * h] = d.x;
            e[2 * h + 1] = d.y;
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) c[m] = fma(m % 4 == 0 ? P.wd[i] : P.ws[i], e[m], c[m]);
    }
    tri_finish(P.swp, c, v);
}

// Position in the channel's order of the triple handled by this wave (the
// XCD-contiguous numbering of xcd_order for kTriWaves waves per workgroup).
__device__ __forceinline__ int tri_order(int n_triples) {
    const int per = gridDim.x / 8;
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
    const int o = __builtin_amdgcn_readfirstlane((xcd * per + slot) * kTriWaves + (int)threadIdx.x / kWave);
    return o < n_triples ? o : -1;
}

// Sum the per-group partials of lanes (g, p) over the groups and write (or
// add) the sixteen components of every pair; red: [16][64] doubles of LDS.
__device__ __forceinline__ void finish_tri(double* red, int lane, int ns, int G, bool act, const double (&acc)[16],
                                           double* __restrict__ dx, long vsz, long out, bool add) {
#pragma unroll
    for (int m = 0; m < 16; ++m) red[m * kWave + lane] = act ? acc[m] : 0.0;
    wave_lds_sync();
    if (lane < ns) {
        for (int m = 0; m < 16; ++m) {
            double t = 0.0;
            for (int gg = 0; gg < G; ++gg) t += red[m * kWave + gg * ns + lane];
            double* d = dx + m * vsz + out * ns + lane;
            if (add) *d += t;
            else *d = t;
        }
    }
}

// ------------------------------------------------- state and packing -

// Initial condition (Eq. 14, Eq. 22): sig = 0, Gamma^{mu nu} = J^{mu nu}/4 for
// mu, nu = x, y, z (coupling9[p * 9 + 3 (mu - 1) + (nu - 1)]), the rest 0.
static __global__ void k_tri_init_state(long n, int nf, int ns, const double* __restrict__ coupling9,
                                        double* __restrict__ x) {
    const long vsz = (long)nf * (nf + 1) / 2 * nf * ns;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (i >= nf) {
            const long j = i - nf;
            const int q = (int)(j / vsz), mu = q / 4, nu = q % 4;
            if (mu > 0 && nu > 0) v = 0.25 * coupling9[((j % vsz) % ns) * 9 + 3 * (mu - 1) + (nu - 1)];
        }
        x[i] = v;
    }
}

// The sixteen strains packed per frequency point, chunk-major: element
// i = point * ns + pair, chunk h (components 2h, 2h + 1) at double2
// (point * 8 + h) * ns + pair.
static __global__ void k_tri_pack(long n, int ns, const double* __restrict__ g, double* __restrict__ gv) {
    double2* o = reinterpret_cast<double2*>(gv);
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const long pt = i / ns;
        const int p = (int)(i % ns);
#pragma unroll
        for (int h = 0; h < 8; ++h) o[(pt * 8 + h) * ns + p] = make_double2(g[(2 * h) * n + i], g[(2 * h + 1) * n + i]);
    }
}

// ------------------------------------------------------- self-energy -

static __global__ void __launch_bounds__(kWave)
k_tri_sigma(FlowArgs A, double lam, const double* __restrict__ x, long nv, double* __restrict__ dsig) {
    __shared__ MeshLds M;
    M.load(A, x, nullptr, threadIdx.x);
    A.w = M.w;
    const int n = blockIdx.x, lane = threadIdx.x;
    const double wn = A.w[n];
    const double* g = x + A.nf;
    // lanes 0..31 take x = +Lambda, lanes 32..63 x = -Lambda; lane r of a half
    // reads pair r, its lane 0 also the on-site exchange term
    const int half = lane >> 5, r = lane & 31;
    const double xx = half == 0 ? lam : -lam;
    double f = 0.0;
    for (int p = r; p < A.ns; p += 32) {
        Plan P;
        make_plan(A.w, A.nf, A.ns, wn + xx, 0.0, wn - xx, 1, 0, P);
        f += 2.0 * (double)A.mult[p] * eval_strain(P, g, A.swap, p, true);
    }
    if (r == 0) {
        // the diagonal components: no transposition or xi xi sign reaches them
        Plan Q;
        make_plan(A.w, A.nf, A.ns, wn + xx, xx - wn, 0.0, 2, 0, Q);
        double e = eval_strain(Q, g, A.swap, 0, true);
        for (int m = 1; m < 4; ++m) e += eval_strain(Q, g + 5 * m * nv, A.swap, 0, false);
        f -= e;
    }
    for (int o = 16; o > 0; o >>= 1) f += __shfl_xor(f, o, kWave);
    const double term = f / (xx - odd_interp(A.w, A.nf, M.sig, xx));
    const double other = __shfl(term, 32, kWave);
    if (lane == 0) dsig[n] = (term + other) * kInvTwoPi;
}

// ------------------------------------------------------------- s, u -

// Per-wave LDS of the s/u kernel: plans [2][kPlanChunk] and node weights,
// later the reduction area [16][64].
struct TriSuLds {
    static constexpr size_t plans() { return (size_t)2 * kPlanChunk * sizeof(Plan); }
    static constexpr size_t wts() { return (size_t)kPlanChunk * sizeof(double); }
    static constexpr size_t red() { return (size_t)16 * kWave * sizeof(double); }
    static constexpr size_t bytes() {
        const size_t a = plans() + wts();
        return ((a > red() ? a : red()) + 31) & ~(size_t)31;
    }
};

// One wave per (s,t,u) triple, lanes (g, p): channel CH = 0 (s) or 2 (u);
// the s launch writes dGamma, the u launch adds.
template <int CH>
static __global__ void __launch_bounds__(kWave * kTriWaves) __attribute__((amdgpu_waves_per_eu(3)))
k_tri_su(FlowArgs A, const double* __restrict__ gv, const int* __restrict__ uo_a, const int* __restrict__ uo_c,
         int n_triples, int swap_copy, double* __restrict__ dx) {
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int nf = A.nf, ns = A.ns, nq = A.nq;
    const Shared sh = load_shared(A, lds_raw, false);
    A.w = sh.w;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    unsigned char* base = lds_raw + SharedLds{nf, ns, A.n_terms}.bytes(false) + wid * TriSuLds::bytes();
    Plan* plan = reinterpret_cast<Plan*>(base);
    double* wts = reinterpret_cast<double*>(base + TriSuLds::plans());
    double* red = reinterpret_cast<double*>(base);
    const int o = tri_order(n_triples);
    if (o < 0) return;
    const int qq = o / nf, it = o % nf;
    const int ia = CH == 0 ? A.su_a[qq] : uo_a[qq];
    const int ic = CH == 0 ? A.su_c[qq] : uo_c[qq];
    const Triple T = make_triple(A.w, nf, ia, it, ic);
    const long vsz = (long)n_triples * ns;
    const __amdgpu_buffer_rsrc_t rv = tri_rsrc(gv, swap_copy ? 2 * vsz : vsz);
    const int G = kWave / ns, g = lane / ns, p = lane % ns;
    const bool act = g < G;
    // the exchanged pair: swap[p], or with spin rotations its pre-rotated copy
    // (the second half of gv)
    const int2 pp = make_int2(16 * p, swap_copy ? kTriElemBytes * (int)vsz + 16 * p : 16 * sh.swap[p]);
    const unsigned hs = 16u * ns;
    const int iv = CH == 0 ? ia : ic;
    const int cnt = A.tab_n[CH * nf + iv];
    const double* tw = A.tab_w + (long)(CH * nf + iv) * nq;
    const double* tg = A.tab_g + (long)(CH * nf + iv) * nq;
    double acc[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) acc[m] = 0.0;
    for (int k0 = 0; k0 < cnt; k0 += kPlanChunk) {
        const int kc = min(kPlanChunk, cnt - k0);
        {
            const int j = lane % kPlanChunk, vec = lane / kPlanChunk;
            if (j < kc) {
                const double om = tw[k0 + j];
                Plan P;
                if (CH == 0)
                    make_plan_tri(A.w, nf, ns, T.s, vec == 0 ? T.w1p - om : om - T.w1,
                                  vec == 0 ? om - T.w2p : om - T.w2, 0, ia, P, &sh.lut);
                else
                    make_plan_tri(A.w, nf, ns, vec == 0 ? T.w1 + om : T.w1p + om, vec == 0 ? om - T.w2p : T.w2 - om,
                                  T.u, 2, ic, P, &sh.lut);
                to_bytes_tri(P);
                plan[vec * kPlanChunk + j] = P;
                if (vec == 0) wts[j] = tg[k0 + j];
            }
        }
        wave_lds_sync();
        if (act) {
            for (int k = g; k < kc; k += G) {
                double a[16], b[16];
                eval_tri(plan[k], rv, pp, hs, a);
                const double W = wts[k];
#pragma unroll
                for (int m = 0; m < 16; ++m) a[m] *= W;
                eval_tri(plan[kPlanChunk + k], rv, pp, hs, b);
                if constexpr (CH == 0) tri_mul<kTriS>(a, b, acc);
                else tri_mul<kTriU>(a, b, acc);
            }
        }
        wave_lds_sync();
    }
    finish_tri(red, lane, ns, G, act, acc, dx + nf, vsz, T.out, CH != 0);
}

// ---------------------------------------------------------------- t -

// Per-wave LDS of the t kernel (ns pairs): plans [2][kTChunk], on-site
// vertices [2][16][kTChunk], node weights, the site vectors of one sub-chunk
// of G = 64/ns nodes (W a and b, [G][16][ns] each: component-major, so the
// lanes of the lattice-sum phase, which read different pairs, hit
// different banks); the two reduction areas [16][64] reuse them.
struct TriTLds {
    int ns;
    __host__ __device__ int G() const { return kWave / ns; }
    __host__ __device__ size_t plans() const { return (size_t)2 * kTChunk * sizeof(Plan); }
    __host__ __device__ size_t ons() const { return (size_t)2 * 16 * kTChunk * sizeof(double); }
    __host__ __device__ size_t wts() const { return (size_t)kTChunk * sizeof(double); }
    __host__ __device__ size_t vec() const { return (size_t)G() * ns * 16 * sizeof(double); }
    __host__ __device__ size_t vbase() const { return plans() + ons() + wts(); }
    __host__ __device__ size_t bytes() const {
        const size_t v = 2 * vec();
        const size_t r = (size_t)2 * 16 * kWave * sizeof(double);     // two reduction areas
        return (vbase() + (v > r ? v : r) + 31) & ~(size_t)31;
    }
};

// One wave per triple, ordered by (t, s, u); adds to dGamma.  Per sub-chunk
// of G nodes, lanes (g, p) interpolate W a and b of node g for pair p into
// LDS and add the two vertex corrections of pair p; then lanes (g, p) run
// over every G-th tabulated term (ka, kb, count) of pair p and add
// count (-2) sum_k Gamma_a^{mu k} Gamma_b^{k nu} for each node.
// ROT: tables with spin rotations (the lattice-sum factors read through
// them; a separate instance, so that the plain one keeps its code).
template <bool ROT>
static __global__ void __launch_bounds__(kWave * kTriWaves) __attribute__((amdgpu_waves_per_eu(2)))
k_tri_t(FlowArgs A, const double* __restrict__ gv, int n_triples, int swap_copy, const int* __restrict__ rpa_rot,
        const int* __restrict__ rot16, int n_rot, const int* __restrict__ seg, const int* __restrict__ seg_off,
        int nseg, double* __restrict__ dx) {
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int nf = A.nf, ns = A.ns, nq = A.nq;
    const Shared sh = load_shared(A, lds_raw, true);
    A.w = sh.w;
    const TriTLds L{ns};
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    // terms' rotations and the rotation tables (spin permutations only)
    const size_t rb0 = SharedLds{nf, ns, A.n_terms}.bytes(true);
    const TriRotLds RL{A.n_terms, ROT ? n_rot : 1};
    int* trot = reinterpret_cast<int*>(lds_raw + rb0);            // [n_terms]
    int* r16 = trot + A.n_terms;                                  // [n_rot][16]
    if (ROT) {
        for (int i = threadIdx.x; i < A.n_terms; i += blockDim.x) trot[i] = rpa_rot[i];
        for (int i = threadIdx.x; i < 16 * n_rot; i += blockDim.x) r16[i] = rot16[i];
        __syncthreads();
    }
    unsigned char* base = lds_raw + rb0 + RL.bytes() + wid * L.bytes();
    Plan* plan = reinterpret_cast<Plan*>(base);                                      // [2][kTChunk]
    double* ons = reinterpret_cast<double*>(base + L.plans());                       // [2][16][kTChunk]
    double* wts = reinterpret_cast<double*>(base + L.plans() + L.ons());             // [kTChunk]
    double* va = reinterpret_cast<double*>(base + L.vbase());                        // [G][16][ns]
    double* vb = va + (size_t)L.G() * ns * 16;                                       // [G][16][ns]
    double* red = va;                                                                // [16][64] corrections
    double* red_s = va + 16 * kWave;                                                 // [16][64] segments
    const int o = tri_order(n_triples);
    if (o < 0) return;
    const int nsu = nf * (nf + 1) / 2;
    const int it = o / nsu, su = o % nsu;
    const Triple T = make_triple(A.w, nf, A.su_a[su], it, A.su_c[su]);
    const double t = T.t;
    const long vsz = (long)n_triples * ns;
    const __amdgpu_buffer_rsrc_t rv = tri_rsrc(gv, swap_copy ? 2 * vsz : vsz);
    const int G = kWave / ns, g = lane / ns, p = lane % ns;
    const bool act = g < G;
    const int2 pp = make_int2(16 * p, swap_copy ? kTriElemBytes * (int)vsz + 16 * p : 16 * sh.swap[p]);
    const int2 p0 = make_int2(0, swap_copy ? kTriElemBytes * (int)vsz : 16 * sh.swap[0]);
    const unsigned hs = 16u * ns;
    const int cnt = A.tab_n[1 * nf + it];
    const double* tw = A.tab_w + (long)(1 * nf + it) * nq;
    const double* tg = A.tab_g + (long)(1 * nf + it) * nq;
    // this lane's segment of the lattice-sum terms
    const bool sact = lane < nseg;
    const int q0 = sact ? seg[2 * lane] : 0, q1 = sact ? seg[2 * lane + 1] : 0;
    double acc[16], accs[16];         // vertex corrections (lanes (g, p)); lattice sum (segments)
#pragma unroll
    for (int m = 0; m < 16; ++m) acc[m] = accs[m] = 0.0;
    for (int k0 = 0; k0 < cnt; k0 += kTChunk) {
        const int kc = min(kTChunk, cnt - k0);
        {
            // lane (role, j): role 0/1 the site-vector plans a/b of node j,
            // role 2/3 the on-site vertices (pair 0) of the two corrections
            const int j = lane % kTChunk, role = lane / kTChunk;
            if (j < kc) {
                const double om = tw[k0 + j];
                const double a0 = role == 0 ? T.w1 + om : (role == 1 ? om + T.w2p : (role == 2 ? T.w2p + om : T.w1 + om));
                const double a1 = role == 0 ? t : (role == 1 ? t : (role == 2 ? T.w2 - om : om - T.w1p));
                const double a2 = role == 0 ? T.w1p - om : (role == 1 ? om - T.w2 : -t);
                Plan P;
                make_plan_tri(A.w, nf, ns, a0, a1, a2, role < 2 ? 1 : 2, it, P, &sh.lut);
                to_bytes_tri(P);
                if (role < 2) {
                    plan[role * kTChunk + j] = P;
                    if (role == 0) wts[j] = tg[k0 + j];
                } else {
                    double v[16];
                    eval_tri(P, rv, p0, hs, v);
#pragma unroll
                    for (int m = 0; m < 16; ++m) ons[((role - 2) * 16 + m) * kTChunk + j] = v[m];
                }
            }
        }
        wave_lds_sync();
        for (int s0 = 0; s0 < kc; s0 += G) {
            const int sc = min(G, kc - s0);
            if (act && g < sc) {
                const int k = s0 + g;
                const double W = wts[k];
                double a[16], h[16];
                eval_tri(plan[k], rv, pp, hs, a);
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    a[m] *= W;
                    va[(g * 16 + m) * ns + p] = a[m];
                    h[m] = ons[(0 * 16 + m) * kTChunk + k];
                }
                tri_mul<kTriC1>(a, h, acc);                 // W (A, O1)
                eval_tri(plan[kTChunk + k], rv, pp, hs, a);     // b
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    vb[(g * 16 + m) * ns + p] = a[m];
                    h[m] = ons[(1 * 16 + m) * kTChunk + k];
                    a[m] *= W;
                }
                tri_mul<kTriC2>(h, a, acc);                 // W (O2, B)
            }
            wave_lds_sync();
            if constexpr (!ROT) {
              {
                for (int qq = q0; qq < q1; ++qq) {
                    const int tq = sh.terms[qq];
                    const int kab = tq & 0xffff, ka = kab / ns, kb = kab % ns;
                    const double cntq = (double)(tq >> 16);
                    for (int kk = 0; kk < sc; ++kk) {
                        double x[16], y[16];
#pragma unroll
                        for (int m = 0; m < 16; ++m) {
                            x[m] = cntq * va[(kk * 16 + m) * ns + ka];
                            y[m] = vb[(kk * 16 + m) * ns + kb];
                        }
                        tri_mul<kTriRpa>(x, y, accs);
                    }
                }
              }
            } else {
                // W_a Gamma_ka W_a^T and W_b Gamma_kb W_b^T (Sec. 4.1)
                for (int qq = q0; qq < q1; ++qq) {
                    const int tq = sh.terms[qq];
                    const int kab = tq & 0xffff, ka = kab / ns, kb = kab % ns;
                    const double cntq = (double)(tq >> 16);
                    const int rw = trot[qq];
                    const int* ra = r16 + 16 * (rw & 0xff);
                    const int* rb = r16 + 16 * (rw >> 8);
                    for (int kk = 0; kk < sc; ++kk) {
                        double x[16], y[16];
                        const double* sa = va + kk * 16 * ns + ka;
                        const double* sb = vb + kk * 16 * ns + kb;
#pragma unroll
                        for (int m = 0; m < 16; ++m) {
                            const int wa = ra[m], wb = rb[m];
                            const double xa = sa[(wa & 15) * ns], yb = sb[(wb & 15) * ns];
                            x[m] = cntq * ((wa & 16) ? -xa : xa);
                            y[m] = (wb & 16) ? -yb : yb;
                        }
                        tri_mul<kTriRpa>(x, y, accs);
                    }
                }
            }
            wave_lds_sync();
        }
    }
    // corrections of lanes (g, p) and segment sums, both to LDS, then pair p
    // adds its node groups and its segments in a fixed order
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        red[m * kWave + lane] = act ? acc[m] : 0.0;
        red_s[m * kWave + lane] = sact ? accs[m] : 0.0;
    }
    wave_lds_sync();
    if (lane < ns) {
        const int s0 = seg_off[lane], s1 = seg_off[lane + 1];
        for (int m = 0; m < 16; ++m) {
            double tsum = 0.0;
            for (int gg = 0; gg < G; ++gg) tsum += red[m * kWave + gg * ns + lane];
            for (int ss = s0; ss < s1; ++ss) tsum += red_s[m * kWave + ss];
            dx[nf + m * vsz + T.out * ns + lane] += tsum;
        }
    }
}

// ------------------------------------------------------ correlations -

// Workgroup (p, slice): the part of the double integrals of pair p over the
// node pairs of its slice, per component m (real parts):
// part[((p * slices + slice) * 16 + m].
static __global__ void __launch_bounds__(kChiThreads)
k_tri_chi_pairs(const double* __restrict__ w, int nf, int ns, const int* __restrict__ swap,
                const double* __restrict__ x, const double* __restrict__ cw, const double* __restrict__ cq,
                const double* __restrict__ cg2, const int* __restrict__ cn, const int* __restrict__ swap_rot,
                const int* __restrict__ rot16, double* __restrict__ part) {
    __shared__ double rr[16][kChiThreads];
    const int p = blockIdx.x, sl = blockIdx.y, tid = threadIdx.x;
    const int n = *cn;
    const long vsz = (long)nf * (nf + 1) / 2 * nf * ns;
    const double* g = x + nf;
    const int nn = n * n;
    const int e0 = (int)((long)nn * sl / kChiSlices), e1 = (int)((long)nn * (sl + 1) / kChiSlices);
    // the exchanged pairs' rotations (spin permutations only)
    const int* wp = rot16 ? rot16 + 16 * swap_rot[p] : nullptr;
    const int* w0 = rot16 ? rot16 + 16 * swap_rot[0] : nullptr;
    double az[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) az[m] = 0.0;
    for (int e = e0 + tid; e < e1; e += kChiThreads) {
        const int i = e / n, j = e % n;
        const double w1 = cw[i], w2 = cw[j];
        const double f = cq[i] * cq[j] * cg2[i] * cg2[j];
        Plan P;
        make_plan_tri(w, nf, ns, w1 + w2, 0.0, w1 - w2, 1, 0, P, nullptr);
        double v[16], tz[16];
        eval_tri_state(P, g, vsz, swap, p, v, wp);
#pragma unroll
        for (int m = 0; m < 16; ++m) tz[m] = tri_ie(m) ? 0.0 : 4.0 * v[m];
        if (p == 0) {
            make_plan_tri(w, nf, ns, w1 + w2, w2 - w1, 0.0, 2, 0, P, nullptr);
            eval_tri_state(P, g, vsz, swap, 0, v, w0);
#pragma unroll
            for (int m = 0; m < 16; ++m)
#pragma unroll
                for (int qp = 0; qp < 16; ++qp)
                    if (tri_chi_x(m, qp) != 0) tz[m] = fma(-(double)tri_chi_x(m, qp), v[qp], tz[m]);
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) az[m] = fma(f, tz[m], az[m]);
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) rr[m][tid] = az[m];
    __syncthreads();
    for (int st = kChiThreads / 2; st > 0; st >>= 1) {
        if (tid < st)
#pragma unroll
            for (int m = 0; m < 16; ++m) rr[m][tid] += rr[m][tid + st];
        __syncthreads();
    }
    if (tid < 16) part[((long)p * kChiSlices + sl) * 16 + tid] = rr[tid][0];
}

// chi[m * ns + p] (m = 4 mu + nu) from the slices, with the on-site one-loop
// term on the diagonal components.
static __global__ void k_tri_chi_final(int ns, const double* __restrict__ cq, const double* __restrict__ cg2,
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
    for (int m = 0; m < 16; ++m) {
        double s = 0.0;
        for (int sl = 0; sl < kChiSlices; ++sl) s += part[((long)p * kChiSlices + sl) * 16 + m];
        chi[m * ns + p] = -pref * s + (m % 5 == 0 ? b : 0.0);
    }
}

}  // namespace pffrg
