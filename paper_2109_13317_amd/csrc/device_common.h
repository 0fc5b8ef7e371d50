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

// An interpolation plan: where the (at most four, see below) contributing
// corners of one vertex evaluation sit in a strain, their weights for the
// spin and the density strain, and whether the two sites are exchanged.
// Every evaluation in the flow has one frequency argument exactly on the
// mesh (or 0, which extrapolates to the first mesh point), so trilinear
// interpolation touches at most four corners.
struct Plan {
    int off[4];       // ((a(a+1)/2 + c) * nf + t) * ns : add the pair index
    double ws[4];     // spin-strain weights
    double wd[4];     // density-strain weights (carry the s<->u signs)
    int n;            // corners in use
    int swp;          // 1: read the exchanged pair swap[p]
};

__device__ __forceinline__ void make_plan(const double* __restrict__ w, int nf, int ns,
                                          double s, double t, double u, Plan& P) {
    int swp = 0;
    double sd = 1.0;
    if (s < 0.0) { s = -s; swp ^= 1; }
    if (t < 0.0) t = -t;
    if (u < 0.0) { u = -u; swp ^= 1; }
    if (s < u) { double q = s; s = u; u = q; sd = -1.0; }
    int sa[2], ta[2], ua[2];
    double fs[2], ft[2], fu[2];
    bracket(w, nf, s, sa[0], sa[1], fs[0], fs[1]);
    bracket(w, nf, t, ta[0], ta[1], ft[0], ft[1]);
    bracket(w, nf, u, ua[0], ua[1], fu[0], fu[1]);
    const int nsn = fs[1] != 0.0 ? 2 : 1;
    const int ntn = ft[1] != 0.0 ? 2 : 1;
    const int nun = fu[1] != 0.0 ? 2 : 1;
    int n = 0;
    for (int iu = 0; iu < nun; ++iu)
        for (int it = 0; it < ntn; ++it)
            for (int is = 0; is < nsn; ++is) {
                double wg = fu[iu] * ft[it] * fs[is];
                int a = sa[is], c = ua[iu];
                double cs = 1.0;
                if (a < c) { int q = a; a = c; c = q; cs = -1.0; }
                if (n < 4) {
                    P.off[n] = (int)((su_index(a, c) * nf + ta[it]) * ns);
                    P.ws[n] = wg;
                    P.wd[n] = sd * cs * wg;
                }
                ++n;
            }
    P.n = n < 4 ? n : 4;
    P.swp = swp;
}

// Value of both strains of pair p through a plan.
__device__ __forceinline__ void eval_plan(const Plan& P, const double* __restrict__ gs,
                                          const double* __restrict__ gd,
                                          const int* __restrict__ swap, int p,
                                          double& vs, double& vd) {
    const int q = P.swp ? swap[p] : p;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < P.n; ++i) {
        a = fma(P.ws[i], gs[P.off[i] + q], a);
        b = fma(P.wd[i], gd[P.off[i] + q], b);
    }
    vs = a;
    vd = b;
}

}  // namespace pffrg
