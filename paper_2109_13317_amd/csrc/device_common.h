// device_common.h -- frequency look-ups shared by the flow kernels.
//
// Conventions (arXiv:2109.13317):
//   * positive mesh w[0..nf), ascending; negative frequencies by symmetry;
//   * Sigma = i sig with sig odd (Eq. 15), linear interpolation between
//     mesh points and constant extrapolation outside (Eq. 36);
//   * vertex strains stored for s >= u >= 0, t >= 0 (Sec. 4.2, Sec. 4.4);
//     other arguments follow from the symmetry relations (Eq. 18, xi of
//     Eq. 19): s -> -s and u -> -u exchange the two sites, t -> -t is free,
//     s <-> u leaves the spin strain and flips the density strain;
//   * interpolation is trilinear (Eq. 37) with constant extrapolation; a
//     corner with s-index < u-index is read through the s <-> u relation.
#pragma once

#include <hip/hip_runtime.h>

namespace pffrg {

constexpr double kInvTwoPi = 0.15915494309189533576888376337251;

__device__ __forceinline__ long su_index(int a, int c) { return (long)a * (a + 1) / 2 + c; }

// Largest mesh index lo with w[lo] <= x and linear weights; constant outside.
__device__ __forceinline__ void bracket(const double* __restrict__ w, int nf, double x,
                                        int& i0, int& i1, double& f0, double& f1) {
    if (x <= w[0]) { i0 = i1 = 0; f0 = 1.0; f1 = 0.0; return; }
    if (x >= w[nf - 1]) { i0 = i1 = nf - 1; f0 = 1.0; f1 = 0.0; return; }
    int lo = 0, hi = nf - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (w[mid] <= x) lo = mid; else hi = mid;
    }
    double h = w[hi] - w[lo];
    i0 = lo; i1 = hi;
    f0 = (w[hi] - x) / h;
    f1 = (x - w[lo]) / h;
}

// Odd function given on the positive mesh (self-energy and its flow).
__device__ __forceinline__ double odd_interp(const double* __restrict__ w, int nf,
                                             const double* __restrict__ v, double x) {
    double sg = 1.0;
    if (x < 0.0) { x = -x; sg = -1.0; }
    int i0, i1; double f0, f1;
    bracket(w, nf, x, i0, i1, f0, f1);
    return sg * (f0 * v[i0] + f1 * v[i1]);
}

// An interpolation plan: where the four contributing corners of one vertex
// evaluation sit in a strain, their weights for the spin and the density
// strain, and whether the two sites are exchanged.  Every evaluation in the
// flow has one frequency argument exactly on the mesh (or 0, which
// extrapolates to the first mesh point), whose slot and mesh index the
// caller passes, so trilinear interpolation touches at most four corners.
// Unused corners repeat a used one with weight 0.
// R is the type the weights are applied in (double, or float in the FP32
// mode); the brackets themselves are always found in FP64.
template <class R>
struct PlanT {
    int off[4];       // element offset ((a(a+1)/2 + c) * nf + t) * ns: add the pair index
    R ws[4];          // spin-strain weights
    R wd[4];          // density-strain weights (carry the s<->u signs)
    int swp;          // 1: read the exchanged pair swap[p]
};
using Plan = PlanT<double>;

// The same plan with the weights left as the two bracket fractions t0, t1 of
// the free slots: corner 2i + j weighs ((1 - t0, t0)[i]) ((1 - t1, t1)[j]),
// formed where the plan is applied.  It is less than half the size of a
// PlanT<double> in LDS and in registers.  flags: bit k set = the density weight
// of corner k is negated (an s <-> u corner), bit 4 = exchanged pair.
struct FracPlan {
    int off[4];
    double t0, t1;
    int flags;
};

// The weights stored into a plan: products of the two bracket weights (and
// the density sign), or the fractions alone.
template <class R>
__device__ __forceinline__ void plan_start(PlanT<R>&) {}
__device__ __forceinline__ void plan_start(FracPlan& P) { P.flags = 0; }
template <class R>
__device__ __forceinline__ void plan_corner(PlanT<R>& P, int k, double g0, double g1, bool neg) {
    const double wg = g0 * g1;
    P.ws[k] = (R)wg;
    P.wd[k] = (R)(neg ? -wg : wg);
}
__device__ __forceinline__ void plan_corner(FracPlan& P, int k, double, double, bool neg) {
    P.flags |= (int)neg << k;
}
template <class R>
__device__ __forceinline__ void plan_finish(PlanT<R>& P, int swp, double, double) {
    P.swp = swp;
}
__device__ __forceinline__ void plan_finish(FracPlan& P, int swp, double t0, double t1) {
    P.flags |= swp << 4;
    P.t0 = t0;
    P.t1 = t1;
}

// Mesh look-up table.  The bits of a positive double, read as an unsigned
// integer, grow with its value, so key(x) = bits(x) >> shift (the exponent
// and the leading mantissa bits) cuts the mesh range into buckets, each a
// fixed fraction of an octave.  lut[key(x) - kmin] is the bracket of the
// smallest value of x's bucket; from there a forward search finds x's own
// bracket in a step or two wherever the mesh holds at most a point or two
// per bucket (the logarithmic meshes of the flow: under one).
constexpr int kLutMax = 512;   // buckets (bytes of LDS)

__host__ __device__ inline unsigned lut_key(double x, int shift) {
    return (unsigned)(__builtin_bit_cast(unsigned long long, x) >> shift);
}

struct MeshLut {
    const double* ih;            // ih[i] = 1 / (w[i+1] - w[i])
    const unsigned char* lut;    // [kLutMax] first bracket of each bucket
    int shift, kmin;
};

// Host: the table of mesh w[0..nf) (positive, ascending, 2 <= nf <= 256):
// the finest key (shift >= 32, so that it fits 32 bits) whose range fits
// kLutMax buckets; per bucket the largest i <= nf - 2 with w[i] <= its
// smallest value (0 below w[0]); buckets past the range hold nf - 2.
inline void build_mesh_lut(const double* w, int nf, unsigned char* lut, int& shift, int& kmin) {
    shift = 32;
    while (shift < 62 && lut_key(w[nf - 1], shift) - lut_key(w[0], shift) >= (unsigned)kLutMax) ++shift;
    kmin = (int)lut_key(w[0], shift);
    const int n = (int)lut_key(w[nf - 1], shift) - kmin + 1;
    int lo = 0;
    for (int b = 0; b < kLutMax; ++b) {
        if (b < n) {
            const double x0 = __builtin_bit_cast(double, (unsigned long long)(kmin + b) << shift);
            while (lo + 1 <= nf - 2 && w[lo + 1] <= x0) ++lo;
            lut[b] = (unsigned char)lo;
        } else {
            lut[b] = (unsigned char)(nf - 2);
        }
    }
}

// Bracket of x >= 0 through the look-up table: the largest lo with
// w[lo] <= x (what a binary search over the mesh finds), weights
// f1 = (x - w[lo]) ih[lo], f0 = 1 - f1; constant outside the mesh.
__host__ __device__ __forceinline__ void bracket_lut(const double* __restrict__ w, const MeshLut& m, int nf,
                                                     double x, int& i0, int& i1, double& f0, double& f1) {
    if (x <= w[0]) { i0 = i1 = 0; f0 = 1.0; f1 = 0.0; return; }
    if (x >= w[nf - 1]) { i0 = i1 = nf - 1; f0 = 1.0; f1 = 0.0; return; }
    // w[0] < x < w[nf-1]: the key lies in the table's range (clamped all
    // the same, so that a NaN stays in bounds; it then leaves lo as found)
    const unsigned k = lut_key(x, m.shift) - (unsigned)m.kmin;
    int lo = m.lut[k < (unsigned)kLutMax ? k : (unsigned)(kLutMax - 1)];
    while (w[lo + 1] <= x) ++lo;   // stops at nf - 2 at the latest: w[nf-1] > x
    i0 = lo; i1 = lo + 1;
    f1 = (x - w[lo]) * m.ih[lo];
    f0 = 1.0 - f1;
}

// kslot in {0,1,2}: which of (s, t, u) holds the on-mesh value, kidx its mesh
// index (0 for a zero argument).  lut: the mesh look-up table (NULL: binary
// search and division).  PL: PlanT<R> or FracPlan.
template <class PL>
__device__ __forceinline__ void make_plan(const double* __restrict__ w, int nf, int ns,
                                          double s, double t, double u, int kslot, int kidx, PL& P,
                                          const MeshLut* lut = nullptr) {
    int swp = 0;
    double sd = 1.0;
    if (s < 0.0) { s = -s; swp ^= 1; }
    if (t < 0.0) t = -t;
    if (u < 0.0) { u = -u; swp ^= 1; }
    if (s < u) {
        const double q = s; s = u; u = q;
        sd = -1.0;
        kslot = kslot == 0 ? 2 : (kslot == 2 ? 0 : 1);
    }
    // the two free slots, in (s, t, u) order, and their brackets
    const int f0 = kslot == 0 ? 1 : 0;
    const int f1 = kslot == 2 ? 1 : 2;
    const double v0 = f0 == 0 ? s : t;
    const double v1 = f1 == 1 ? t : u;
    int b0[2], b1[2];
    double g0[2], g1[2];
    plan_start(P);
    if (lut) {
        bracket_lut(w, *lut, nf, v0, b0[0], b0[1], g0[0], g0[1]);
        bracket_lut(w, *lut, nf, v1, b1[0], b1[1], g1[0], g1[1]);
    } else {
        bracket(w, nf, v0, b0[0], b0[1], g0[0], g0[1]);
        bracket(w, nf, v1, b1[0], b1[1], g1[0], g1[1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int ia = kslot == 0 ? kidx : b0[i];
            const int it = kslot == 1 ? kidx : (kslot == 0 ? b0[i] : b1[j]);
            const int ic = kslot == 2 ? kidx : b1[j];
            int a = ia, c = ic;
            double cs = sd;
            if (a < c) { const int q = a; a = c; c = q; cs = -cs; }
            P.off[2 * i + j] = (int)((su_index(a, c) * nf + it) * ns);
            plan_corner(P, 2 * i + j, g0[i], g1[j], cs < 0.0);
        }
    plan_finish(P, swp, g0[1], g1[1]);
}

// Value of both strains of pair p through a plan.
__device__ __forceinline__ void eval_plan(const Plan& P, const double* __restrict__ gs,
                                          const double* __restrict__ gd,
                                          const int* __restrict__ swap, int p,
                                          double& vs, double& vd) {
    const int q = P.swp ? swap[p] : p;
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        a = fma(P.ws[i], gs[P.off[i] + q], a);
        b = fma(P.wd[i], gd[P.off[i] + q], b);
    }
    vs = a;
    vd = b;
}

}  // namespace pffrg
