// kernels_obs.h -- correlations and Runge-Kutta vector kernels.
//
// Correlations (arXiv:2109.13317, Eq. 30, contracted with Eq. 25 for SU(2)):
//   chi^{zz}_{ij} = d_ij/(4pi) I g^2 - 1/(16pi^2) II g1^2 g2^2
//        [4 Gs_ij(w1+w2, 0, w1-w2) + d_ij (2 Gs_ii - 2 Gd_ii)(w1+w2, w2-w1, 0)]
//   chi^{00}_{ij} = d_ij/(4pi) I g^2 - 1/(16pi^2) II g1^2 g2^2
//        [4 Gd_ij(w1+w2, 0, w1-w2) - d_ij (6 Gs_ii + 2 Gd_ii)(w1+w2, w2-w1, 0)]
// with g = 1/(w - sig(w)) on |w| >= Lambda (G = -i g), trapezoid on the mesh
// points of [-wmax, -Lambda] and [Lambda, wmax] plus the ends, tensor
// product in two dimensions.  chi(k) is Eq. 31 normalised per unit cell.
#pragma once

#include "device_common.h"

namespace pffrg {

constexpr int kMaxMesh = 128;     // largest mesh (LDS copies)

// One wave: nodes, trapezoid weights and g^2 of the correlation integrals
// (mesh and self-energy staged in LDS; lanes fill the node list).
static __global__ void __launch_bounds__(64)
k_chi_nodes(const double* __restrict__ w, int nf, double lam, const double* __restrict__ x,
            double* __restrict__ cw, double* __restrict__ cq, double* __restrict__ cg2, int* __restrict__ cn) {
    __shared__ double sw[kMaxMesh], ss[kMaxMesh];
    const int lane = threadIdx.x;
    for (int i = lane; i < nf; i += 64) { sw[i] = w[i]; ss[i] = x[i]; }
    __syncthreads();
    const double wmax = sw[nf - 1];
    const double lo2[2] = {-wmax, lam}, hi2[2] = {-lam, wmax};
    int n = 0;
    for (int q = 0; q < 2; ++q) {
        const double lo = lo2[q], hi = hi2[q];
        if (!(lo < hi)) continue;
        // mesh points inside (lo, hi): a contiguous run of the full mesh
        int below = 0, cnt = 0;
        for (int i = lane; i < 2 * nf; i += 64) {
            const double v = i < nf ? -sw[nf - 1 - i] : sw[i - nf];
            below += v <= lo;
            cnt += (v > lo && v < hi);
        }
        for (int o = 32; o > 0; o >>= 1) {
            below += __shfl_xor(below, o, 64);
            cnt += __shfl_xor(cnt, o, 64);
        }
        const int m = cnt + 2;
        for (int j = lane; j < m; j += 64) {
            auto node = [&](int jj) {
                if (jj == 0) return lo;
                if (jj == m - 1) return hi;
                const int i = below + jj - 1;
                return i < nf ? -sw[nf - 1 - i] : sw[i - nf];
            };
            const double cur = node(j);
            const double wl = j > 0 ? 0.5 * (cur - node(j - 1)) : 0.0;
            const double wr = j + 1 < m ? 0.5 * (node(j + 1) - cur) : 0.0;
            cw[n + j] = cur;
            cq[n + j] = wl + wr;
            const double g = 1.0 / (cur - odd_interp(sw, nf, ss, cur));
            cg2[n + j] = g * g;
        }
        n += m;
    }
    if (lane == 0) *cn = n;
}

constexpr int kChiThreads = 256;

// Workgroup (p, slice): the part of the double integral of pair p over the
// node pairs e = (i, j) of its slice; part[(p * slices + slice) * 2 + {0,1}].
constexpr int kChiSlices = 16;

static __global__ void __launch_bounds__(kChiThreads)
k_chi_pairs(const double* __restrict__ w, int nf, int ns, const int* __restrict__ swap,
            const double* __restrict__ x, const double* __restrict__ cw,
            const double* __restrict__ cq, const double* __restrict__ cg2,
            const int* __restrict__ cn, double* __restrict__ part) {
    __shared__ double rz[kChiThreads], rd[kChiThreads];
    const int p = blockIdx.x, sl = blockIdx.y, tid = threadIdx.x;
    const int n = *cn;
    const long vsz = (long)nf * (nf + 1) / 2 * nf * ns;
    const double* gs = x + nf;
    const double* gd = gs + vsz;
    const int nn = n * n;
    const int e0 = (int)((long)nn * sl / kChiSlices), e1 = (int)((long)nn * (sl + 1) / kChiSlices);
    double az = 0.0, ad = 0.0;
    for (int e = e0 + tid; e < e1; e += kChiThreads) {
        const int i = e / n, j = e % n;
        const double w1 = cw[i], w2 = cw[j];
        const double f = cq[i] * cq[j] * cg2[i] * cg2[j];
        Plan P;
        make_plan(w, nf, ns, w1 + w2, 0.0, w1 - w2, 1, 0, P);
        double vs, vd;
        eval_plan(P, gs, gd, swap, p, vs, vd);
        double tz = 4.0 * vs, td = 4.0 * vd;
        if (p == 0) {
            make_plan(w, nf, ns, w1 + w2, w2 - w1, 0.0, 2, 0, P);
            double es, ed;
            eval_plan(P, gs, gd, swap, 0, es, ed);
            tz += 2.0 * es - 2.0 * ed;
            td -= 6.0 * es + 2.0 * ed;
        }
        az = fma(f, tz, az);
        ad = fma(f, td, ad);
    }
    rz[tid] = az;
    rd[tid] = ad;
    __syncthreads();
    for (int st = kChiThreads / 2; st > 0; st >>= 1) {
        if (tid < st) { rz[tid] += rz[tid + st]; rd[tid] += rd[tid + st]; }
        __syncthreads();
    }
    if (tid == 0) {
        part[(p * kChiSlices + sl) * 2 + 0] = rz[0];
        part[(p * kChiSlices + sl) * 2 + 1] = rd[0];
    }
}

// chi[p], chi[ns + p] from the slices, with the on-site one-loop term.
static __global__ void k_chi_final(int ns, const double* __restrict__ cq, const double* __restrict__ cg2,
                                   const int* __restrict__ cn, const double* __restrict__ part,
                                   double* __restrict__ chi) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ns) return;
    double sz = 0.0, sd = 0.0;
    for (int sl = 0; sl < kChiSlices; ++sl) {
        sz += part[(p * kChiSlices + sl) * 2 + 0];
        sd += part[(p * kChiSlices + sl) * 2 + 1];
    }
    const double pref = 1.0 / (16.0 * M_PI * M_PI);
    double z = -pref * sz, d = -pref * sd;
    if (p == 0) {
        double b = 0.0;
        for (int i = 0; i < *cn; ++i) b = fma(cq[i], cg2[i], b);
        b *= 0.5 * kInvTwoPi;        // 1/(4 pi)
        z += b;
        d += b;
    }
    chi[p] = z;
    chi[ns + p] = d;
}

// The correlations per reduced pair spread onto the layout of the paper's
// observable files (Sec. 5, output data): out[(m * nbs) + k] = chi[m * ns +
// site_pair[k]] for the nbs = n_basis * n_sites_total (basis site, site)
// slots, NaN where a basis site lists fewer sites (site_pair = -1).
static __global__ void k_chi_sites(int nc, int ns, int nbs, const int* __restrict__ site_pair,
                                   const double* __restrict__ chi, double* __restrict__ out) {
    const long n = (long)nc * nbs;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int m = (int)(i / nbs), k = (int)(i % nbs);
        const int sp = site_pair[k];
        out[i] = sp >= 0 ? chi[m * ns + sp] : __builtin_nan("");
    }
}

// chi(k_q) = (1/nb) sum_{b, j} cos(k_q . dr_bj) scale (sum_m chi^m_{pair(b,j)}),
// the sum over the nsum strains chi[m * stride + pair], m < nsum (SU(2): 3
// chi^{zz}; XYZ: chi^xx + chi^yy + chi^zz); one wave per k point, lanes over
// the (basis, site) terms.
constexpr int kChiKWaves = 4;
static __global__ void __launch_bounds__(64 * kChiKWaves)
k_chi_k(int nterm, const int* __restrict__ pair, const double* __restrict__ dr, double inv_nb,
        const double* __restrict__ chi, int nsum, int stride, double scale, int nk, const double* __restrict__ kp,
        double* __restrict__ out) {
    const int q = blockIdx.x * kChiKWaves + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (q >= nk) return;
    const double kx = kp[3 * q], ky = kp[3 * q + 1], kz = kp[3 * q + 2];
    double acc = 0.0;
    for (int i = lane; i < nterm; i += 64) {
        const double ph = kx * dr[3 * i] + ky * dr[3 * i + 1] + kz * dr[3 * i + 2];
        double v = chi[pair[i]];
        for (int m = 1; m < nsum; ++m) v += chi[m * stride + pair[i]];
        acc = fma(cos(ph), v, acc);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) out[q] = scale * inv_nb * acc;
}

// ------------------------------------------------------- Runge-Kutta ----

// y = x + a*k  and  acc = (init ? x : acc) + b*k, one pass over the state.
static __global__ void k_rk_stage(long n, const double* __restrict__ x, const double* __restrict__ k,
                           double a, double* __restrict__ y, double b, double* __restrict__ acc,
                           int init) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double ki = k[i], xi = x[i];
        if (y) y[i] = xi + a * ki;
        if (acc) acc[i] = (init ? xi : acc[i]) + b * ki;
    }
}

// y = x + sum_j c_j k_j for up to 7 stage vectors (c_j == 0 skipped).
struct Combo {
    const double* k[7];
    double c[7];
    int m;
};

static __global__ void k_combine(long n, const double* __restrict__ x, Combo C, double* __restrict__ y) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double v = x ? x[i] : 0.0;
        for (int j = 0; j < C.m; ++j)
            if (C.c[j] != 0.0) v += C.c[j] * C.k[j][i];
        y[i] = v;
    }
}

// Per-block partial reductions for the step control:
//   part[2b]   = max_i |e_i| / (atol + rtol * max(|x_i|, |y_i|))  (e may be NULL -> 0)
//   part[2b+1] = 1 if any x_i or y_i is not finite
constexpr int kRedThreads = 256;
static __global__ void __launch_bounds__(kRedThreads)
k_err_norm(long n, const double* __restrict__ x, const double* __restrict__ y,
           const double* __restrict__ e, double atol, double rtol, double* __restrict__ part) {
    __shared__ double sm[kRedThreads], sf[kRedThreads];
    double m = 0.0, bad = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double yi = y[i];
        const double xi = x ? x[i] : yi;
        if (!isfinite(yi) || !isfinite(xi)) bad = 1.0;
        if (e) {
            const double sc = atol + rtol * fmax(fabs(xi), fabs(yi));
            m = fmax(m, fabs(e[i]) / sc);
        }
    }
    sm[threadIdx.x] = m;
    sf[threadIdx.x] = bad;
    __syncthreads();
    for (unsigned st = kRedThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + st]);
            sf[threadIdx.x] = fmax(sf[threadIdx.x], sf[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = sm[0]; part[2 * blockIdx.x + 1] = sf[0]; }
}

// one wave
static __global__ void __launch_bounds__(64)
k_err_final(int nb, const double* __restrict__ part, double* __restrict__ out) {
    if (blockIdx.x != 0) return;
    const int lane = threadIdx.x;
    double m = 0.0, bad = 0.0;
    for (int b = lane; b < nb; b += 64) { m = fmax(m, part[2 * b]); bad = fmax(bad, part[2 * b + 1]); }
    for (int o = 32; o > 0; o >>= 1) {
        m = fmax(m, __shfl_xor(m, o, 64));
        bad = fmax(bad, __shfl_xor(bad, o, 64));
    }
    if (lane == 0) {
        out[0] = m;
        out[1] = bad;
    }
}

static __global__ void k_init_state(long n, int nf, int ns, const double* __restrict__ coupling,
                             double* __restrict__ x) {
    const long vsz = (long)nf * (nf + 1) / 2 * nf * ns;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (i >= nf && i < nf + vsz) v = 0.25 * coupling[(i - nf) % ns];
        x[i] = v;
    }
}

}  // namespace pffrg
