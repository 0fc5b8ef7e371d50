/*
 * pffrg_oracle.c -- plain, slow, FP64 reference implementation of the SU(2)
 * pseudofermion-FRG flow right-hand side and two-spin correlations.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code, header or table with the GPU library.
 *
 * What it computes, with the passage of arXiv:2109.13317 that defines it:
 *   - Self-energy flow, Sec. 3 explicit one-particle flow (Eq. 23), with the
 *     single-scale propagator S (Eq. 12) collapsing the frequency integral to
 *     the two points |w| = Lambda.
 *   - Vertex flow, Sec. 3 explicit two-particle flow (Eq. 24): s, t (RPA plus
 *     two vertex corrections) and u channels, Katanin propagator (Eq. 13).
 *   - SU(2) vertex (nc = 2 strains): Gamma^{11}=Gamma^{22}=Gamma^{33}
 *     ("spin" strain) and Gamma^{00} ("density" strain), other components
 *     zero (Sec. 3, SU(2) constraint).  XYZ vertex (nc = 4 strains, Sec. 3:
 *     only the diagonal components mu = nu are non-zero): Gamma^{11},
 *     Gamma^{22}, Gamma^{33} (x, y, z) and Gamma^{00} (density).  The density
 *     strain is the last one in both.  The spin contractions of Eq. 24 with
 *     Eq. 25 are done by hand; the coefficients are Pauli-algebra results
 *     (sigma^a sigma^b = delta_ab + i eps_abc sigma^c), and the SU(2) ones are
 *     the XYZ ones with the three spin strains equal.
 *   - TRI vertex (nc = 16 strains, Sec. 3 general time-reversal invariant
 *     case): every Gamma^{mu nu}, index 4 mu + nu, real or imaginary by
 *     Eq. 18 and held as a real number; the channel products, the
 *     self-energy sums and the correlations are evaluated with explicit
 *     spin tensors (Eq. 25) instead of hand-contracted coefficients.
 *   - Vertex symmetries (Eq. 18 with xi of Eq. 19), octant storage s>=u,
 *     t>=0 (Sec. 4.2) and trilinear interpolation with constant
 *     extrapolation (Eq. 37); Sigma odd with linear interpolation (Eq. 36).
 *   - Lattice: translations only.  For every basis site b the vertex is kept
 *     for every site within the bond-distance truncation range (Eq. 34);
 *     no point-group reduction is used, so the oracle trusts no symmetry
 *     table.  Lattice sums run over every site in range of both ends.
 *   - Correlations chi^{zz} and chi^{00} (Eq. 30); TRI: every chi^{mu nu}.
 *
 * Readings where the paper is silent (also listed in the design notes):
 *   R1 (delta parts) S and the S-part of S_kat are integrated analytically at
 *      w = +-Lambda; only the Katanin part -G^2 dSigma/dLambda is integrated
 *      numerically.
 *   R2 (quadrature) the Katanin integral runs over
 *      D = {|w| >= Lambda, |partner(w)| >= Lambda} within [-wmax, wmax];
 *      nodes are the finite endpoints of each connected piece of D plus every
 *      mesh point +-w_n strictly inside it; trapezoid rule inside each piece
 *      (Sec. 4.2: trapezoid nodes coincide with the mesh).  Same rule for the
 *      correlation integrals, tensor-product in two dimensions.
 *   R3 (theta ties) inside D the step function is 1 at its edge; a
 *      propagator G evaluated at a delta point with |argument| == Lambda
 *      exactly takes theta = 1/2.
 *   R4 interpolation corners with s < u are read through the s<->u relation.
 *   R5 chi: the one-loop term carries delta_ij.
 *
 * Real form.  Sigma = i*sig with sig real and odd (Eq. 15).  With
 * g(w) = theta(|w|-Lambda)/(w - sig(w)) one has G = -i g, and the channel
 * bubble [G(w) Skat(p) + G(p) Skat(w)] is real:
 *   -g(w) d(|p|-L)/(p - sig(p)) - g(p) d(|w|-L)/(w - sig(w))
 *   + g(w) g(p)^2 sig'(p) + g(p) g(w)^2 sig'(w).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559
#define MAXC 16   /* most vertex strains per element (TRI) */

typedef struct {
    int nf;              /* number of positive mesh frequencies */
    const double *w;     /* ascending positive mesh, nf entries */
    int nb;              /* basis sites */
    int ns;              /* padded length of each basis site's site list */
    const int *nsites;   /* [nb] sites within range of basis site b */
    const int *cell;     /* [nb][ns][3] cell offset of each listed site */
    const int *bas;      /* [nb][ns]   basis index of each listed site */
    int rm;              /* half-width of the offset lookup box */
    const int *lookup;   /* [nb][2rm+1][2rm+1][2rm+1][nb] -> list index or -1 */
    int nc;              /* vertex strains: 2 (SU(2): spin, density), 4 (XYZ: x, y, z, density), 16 (TRI) */
} orc_lattice;

/* ------------------------------------------------------------ layout --- */

static long su_index(int a, int c) { return (long)a * (a + 1) / 2 + c; }

static long n_su(const orc_lattice *L) { return su_index(L->nf, 0); }

/* Offset of strain `comp` in the state vector (SU(2): 0 spin, 1 density;
 * XYZ: 0 x, 1 y, 2 z, 3 density). */
static long strain_offset(const orc_lattice *L, int comp)
{
    return L->nf + (long)comp * L->nb * n_su(L) * L->nf * L->ns;
}

long orc_state_size(const orc_lattice *L)
{
    return L->nf + (long)L->nc * L->nb * n_su(L) * L->nf * L->ns;
}

/* The density strain Gamma^{00} is the last one; it alone changes sign under s <-> u. */
static int is_density(const orc_lattice *L, int comp) { return comp == L->nc - 1; }

/* Index of vertex value (comp, basis b, s-index a, t-index t, u-index c, site k), a>=c. */
static long vidx(const orc_lattice *L, int comp, int b, int a, int t, int c, int k)
{
    return strain_offset(L, comp) + (((long)b * n_su(L) + su_index(a, c)) * L->nf + t) * L->ns + k;
}

/* --------------------------------------------------------- lattice ----- */

static int site_of(const orc_lattice *L, int b1, const int d[3], int b2)
{
    int W = 2 * L->rm + 1;
    for (int i = 0; i < 3; ++i)
        if (d[i] < -L->rm || d[i] > L->rm) return -1;
    long idx = ((((long)b1 * W + (d[0] + L->rm)) * W + (d[1] + L->rm)) * W + (d[2] + L->rm)) * L->nb + b2;
    return L->lookup[idx];
}

/* ---------------------------------------------------- interpolation ---- */

/* Bracketing mesh points and weights of x >= 0, constant outside the mesh. */
static void bracket(const orc_lattice *L, double x, int *i0, int *i1, double *f0, double *f1)
{
    const double *w = L->w;
    int n = L->nf;
    if (x <= w[0]) { *i0 = *i1 = 0; *f0 = 1.0; *f1 = 0.0; return; }
    if (x >= w[n - 1]) { *i0 = *i1 = n - 1; *f0 = 1.0; *f1 = 0.0; return; }
    int lo = 0;
    while (w[lo + 1] <= x) ++lo;
    double h = w[lo + 1] - w[lo];
    *i0 = lo; *i1 = lo + 1;
    *f0 = (w[lo + 1] - x) / h;
    *f1 = (x - w[lo]) / h;
}

/* Odd function of frequency given on the positive mesh (Eq. 15, Eq. 36). */
static double odd_interp(const orc_lattice *L, const double *v, double x)
{
    double sgn = 1.0;
    if (x < 0.0) { x = -x; sgn = -1.0; }
    int i0, i1; double f0, f1;
    bracket(L, x, &i0, &i1, &f0, &f1);
    return sgn * (f0 * v[i0] + f1 * v[i1]);
}

/*
 * Vertex strain `comp` between site (b1, cell 0) and site (b2, cell d) at
 * transfer frequencies (s,t,u).  Eq. 18 with xi(0)=+1, xi(3)=-1:
 *   s -> -s swaps the two sites; t -> -t is free; u -> -u swaps the sites;
 *   s <-> u is free for the spin strains and flips the density strain.
 * Outside the truncation range the vertex is zero (Eq. 34).
 */
static double vertex(const orc_lattice *L, const double *x, int comp,
                     int b1, const int dR[3], int b2, double s, double t, double u)
{
    int d[3] = {dR[0], dR[1], dR[2]};
    double sign = 1.0;
    if (s < 0.0) { s = -s; int tb = b1; b1 = b2; b2 = tb; d[0] = -d[0]; d[1] = -d[1]; d[2] = -d[2]; }
    if (t < 0.0) t = -t;
    if (u < 0.0) { u = -u; int tb = b1; b1 = b2; b2 = tb; d[0] = -d[0]; d[1] = -d[1]; d[2] = -d[2]; }
    if (s < u) { double q = s; s = u; u = q; if (is_density(L, comp)) sign = -sign; }
    int k = site_of(L, b1, d, b2);
    if (k < 0) return 0.0;

    int sa[2], ta[2], ua[2];
    double fs[2], ft[2], fu[2];
    bracket(L, s, &sa[0], &sa[1], &fs[0], &fs[1]);
    bracket(L, t, &ta[0], &ta[1], &ft[0], &ft[1]);
    bracket(L, u, &ua[0], &ua[1], &fu[0], &fu[1]);
    double acc = 0.0;
    for (int iu = 0; iu < 2; ++iu)
        for (int it = 0; it < 2; ++it)
            for (int is = 0; is < 2; ++is) {
                double wgt = fu[iu] * ft[it] * fs[is];
                if (wgt == 0.0) continue;
                int a = sa[is], c = ua[iu];
                double v;
                if (a >= c) v = x[vidx(L, comp, b1, a, ta[it], c, k)];
                else v = (is_density(L, comp) ? -1.0 : 1.0) * x[vidx(L, comp, b1, c, ta[it], a, k)];
                acc += wgt * v;
            }
    return sign * acc;
}

/* ----------------------------------------------------- propagators ---- */

typedef struct {
    const orc_lattice *L;
    const double *x;       /* state */
    const double *dsig;    /* d sig / d Lambda on the positive mesh */
    double lam;
} orc_eval;

static double sig_at(const orc_eval *E, double w) { return odd_interp(E->L, E->x, w); }
static double dsig_at(const orc_eval *E, double w) { return odd_interp(E->L, E->dsig, w); }

/* 1/(w - sig(w)): the dressed propagator without its step function. */
static double gbare(const orc_eval *E, double w) { return 1.0 / (w - sig_at(E, w)); }

/* Step function at a delta point: 1 outside, 1/2 exactly on the edge (R3). */
static double theta_half(double y, double lam)
{
    double a = fabs(y);
    if (a > lam) return 1.0;
    if (a == lam) return 0.5;
    return 0.0;
}

/* ----------------------------------------------------- quadrature ----- */

#define MAXPIECE 3

/*
 * Connected pieces of D = [-wmax, wmax] minus (-lam, lam) minus (c-lam, c+lam)
 * (R2).  c is the frequency where the partner propagator's argument vanishes.
 */
static int pieces(double c, double lam, double wmax, double lo[MAXPIECE], double hi[MAXPIECE])
{
    double a0[2] = {-wmax, lam}, b0[2] = {-lam, wmax};
    double e0 = c - lam, e1 = c + lam;
    int n = 0;
    for (int i = 0; i < 2; ++i) {
        double a = a0[i], b = b0[i];
        if (!(a < b)) continue;
        double l1 = a, h1 = (b < e0 ? b : e0);
        double l2 = (a > e1 ? a : e1), h2 = b;
        if (l1 < h1) { lo[n] = l1; hi[n] = h1; ++n; }
        if (l2 < h2) { lo[n] = l2; hi[n] = h2; ++n; }
    }
    return n;
}

/* Sorted nodes of one piece: lo, every +-w_n strictly inside, hi. */
static int piece_nodes(const orc_lattice *L, double lo, double hi, double *nodes)
{
    int n = 0;
    nodes[n++] = lo;
    for (int i = L->nf - 1; i >= 0; --i) {
        double v = -L->w[i];
        if (v > lo && v < hi) nodes[n++] = v;
    }
    for (int i = 0; i < L->nf; ++i) {
        double v = L->w[i];
        if (v > lo && v < hi) nodes[n++] = v;
    }
    nodes[n++] = hi;
    return n;
}

/* ------------------------------------------------------- sigma flow --- */

/*
 * d sig/dLambda(w) = (1/2pi) sum_{x=+-Lambda} F(w,x) / (x - sig(x)) with
 *   SU(2): F = 2 sum_j Gd_{0j}(w+x, 0, w-x) - (3 Gs_{00} + Gd_{00})(w+x, x-w, 0)
 *   XYZ:   F = 2 sum_j Gd_{0j}(w+x, 0, w-x) - (Gx + Gy + Gz + Gd)_{00}(w+x, x-w, 0)
 *   TRI:   F from the spin tensors themselves (sigma_sum_tri)
 * (Eq. 23 contracted with Eq. 25: the direct term traces the density
 * strain, the exchange term sums every diagonal component; the sum over j
 * covers every site in range of the reference site, basis site 0).
 */
static double sigma_sum_tri(const orc_lattice *L, const double *x, double w, double xx);

double orc_sigma_rhs_at(const orc_lattice *L, double lam, const double *x, double w)
{
    orc_eval E = {L, x, NULL, lam};
    const int zero[3] = {0, 0, 0};
    const int dens = L->nc - 1;
    double acc = 0.0;
    for (int sx = 0; sx < 2; ++sx) {
        double xx = sx == 0 ? lam : -lam;
        if (L->nc == 16) {
            acc += sigma_sum_tri(L, x, w, xx) / (xx - sig_at(&E, xx));
            continue;
        }
        double f = 0.0;
        for (int k = 0; k < L->nsites[0]; ++k) {
            const int *cr = &L->cell[(long)k * 3];
            f += 2.0 * vertex(L, x, dens, 0, cr, L->bas[k], w + xx, 0.0, w - xx);
        }
        if (L->nc == 2) {
            f -= 3.0 * vertex(L, x, 0, 0, zero, 0, w + xx, xx - w, 0.0);
        } else {
            for (int c = 0; c < 3; ++c) f -= vertex(L, x, c, 0, zero, 0, w + xx, xx - w, 0.0);
        }
        f -= vertex(L, x, dens, 0, zero, 0, w + xx, xx - w, 0.0);
        acc += f / (xx - sig_at(&E, xx));
    }
    return acc / TWO_PI;
}

void orc_sigma_rhs(const orc_lattice *L, double lam, const double *x, double *dsig)
{
    for (int n = 0; n < L->nf; ++n) dsig[n] = orc_sigma_rhs_at(L, lam, x, L->w[n]);
}

/* ------------------------------------------------------ vertex flow --- */

typedef struct {
    int b, k;            /* output pair: basis site b at cell 0, listed site k */
    int bk;              /* basis index of site k */
    int dk[3];           /* cell offset of site k */
    double s, t, u;      /* transfer frequencies */
    double w1p, w2p, w1, w2;   /* external frequencies (Eq. 17 inverted) */
} orc_out;

/* The channel integrands for one frequency w of the loop, already
 * multiplied by `wt`, added to acc[comp] for every strain.
 *
 * SU(2) (acc[0] spin, acc[1] density; A, B the two vertices of each
 * product in the order of Eq. 24):
 *   s: dGs = -2 As Bs + As Bd + Ad Bs,  dGd = 3 As Bs + Ad Bd
 *   u: dGs = +2 As Bs + As Bd + Ad Bs,  dGd = 3 As Bs + Ad Bd
 *   t: dGs = -2 sum_j a_js b_js - As O1s + As O1d - O2s Bs + O2d Bs
 *      dGd = -2 sum_j a_jd b_jd + 3 Ad O1s + Ad O1d + 3 O2s Bd + O2d Bd
 * XYZ (acc[0..2] = x, y, z, acc[3] = density; (a, b, c) any cyclic
 * permutation of (x, y, z), d the density strain):
 *   s: dGd = Ad Bd + Ax Bx + Ay By + Az Bz,  dGa = Ad Ba + Aa Bd - Ab Bc - Ac Bb
 *   u: dGd = Ad Bd + Ax Bx + Ay By + Az Bz,  dGa = Ad Ba + Aa Bd + Ab Bc + Ac Bb
 *   t: dGm = -2 sum_j a_jm b_jm + Am sum_n e(m,n) O1n + Bm sum_n e(m,n) O2n
 *      with e(m,n) = +1 if m or n is the density strain or m = n, else -1.
 */
static void integrand_s(const orc_eval *E, const orc_out *o, double w, double wt, double *acc)
{
    const orc_lattice *L = E->L;
    double A[4], B[4];
    for (int c = 0; c < L->nc; ++c) {
        A[c] = vertex(L, E->x, c, o->b, o->dk, o->bk, o->s, o->w1p - w, w - o->w2p);
        B[c] = vertex(L, E->x, c, o->b, o->dk, o->bk, o->s, w - o->w1, w - o->w2);
    }
    if (L->nc == 2) {
        acc[0] += wt * (-2.0 * A[0] * B[0] + A[0] * B[1] + A[1] * B[0]);
        acc[1] += wt * (3.0 * A[0] * B[0] + A[1] * B[1]);
    } else {
        acc[3] += wt * (A[3] * B[3] + A[0] * B[0] + A[1] * B[1] + A[2] * B[2]);
        acc[0] += wt * (A[3] * B[0] + A[0] * B[3] - A[1] * B[2] - A[2] * B[1]);
        acc[1] += wt * (A[3] * B[1] + A[1] * B[3] - A[2] * B[0] - A[0] * B[2]);
        acc[2] += wt * (A[3] * B[2] + A[2] * B[3] - A[0] * B[1] - A[1] * B[0]);
    }
}

/* e(m,n) of the XYZ t-channel vertex corrections and correlations. */
static double xyz_sign(int m, int n) { return (m == 3 || n == 3 || m == n) ? 1.0 : -1.0; }

static void integrand_t(const orc_eval *E, const orc_out *o, double w, double wt, double *acc)
{
    const orc_lattice *L = E->L;
    const int zero[3] = {0, 0, 0};
    const int nc = L->nc;
    /* particle-hole RPA term: -sum_j Gamma_{i1 j} Gamma_{j i2}, j in range of both */
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < L->nsites[o->b]; ++j) {
        const int *cj = &L->cell[((long)o->b * L->ns + j) * 3];
        int bj = L->bas[(long)o->b * L->ns + j];
        int d2[3] = {o->dk[0] - cj[0], o->dk[1] - cj[1], o->dk[2] - cj[2]};
        if (site_of(L, bj, d2, o->bk) < 0) continue;
        for (int c = 0; c < nc; ++c)
            r[c] += vertex(L, E->x, c, o->b, cj, bj, o->w1 + w, o->t, o->w1p - w)
                  * vertex(L, E->x, c, bj, d2, o->bk, w + o->w2p, o->t, w - o->w2);
    }
    /* vertex corrections with the on-site vertex at i2 and at i1 */
    double A[4], O1[4], O2[4], B[4];
    for (int c = 0; c < nc; ++c) {
        A[c] = vertex(L, E->x, c, o->b, o->dk, o->bk, o->w1 + w, o->t, o->w1p - w);
        O1[c] = vertex(L, E->x, c, o->bk, zero, o->bk, o->w2p + w, o->w2 - w, -o->t);
        O2[c] = vertex(L, E->x, c, o->b, zero, o->b, o->w1 + w, w - o->w1p, -o->t);
        B[c] = vertex(L, E->x, c, o->b, o->dk, o->bk, w + o->w2p, o->t, w - o->w2);
    }
    if (nc == 2) {
        double gs = -2.0 * r[0] - A[0] * O1[0] + A[0] * O1[1] - O2[0] * B[0] + O2[1] * B[0];
        double gd = -2.0 * r[1] + 3.0 * A[1] * O1[0] + A[1] * O1[1] + 3.0 * O2[0] * B[1] + O2[1] * B[1];
        acc[0] += wt * gs;
        acc[1] += wt * gd;
    } else {
        for (int m = 0; m < 4; ++m) {
            double c1 = 0.0, c2 = 0.0;
            for (int n = 0; n < 4; ++n) {
                c1 += xyz_sign(m, n) * O1[n];
                c2 += xyz_sign(m, n) * O2[n];
            }
            acc[m] += wt * (-2.0 * r[m] + A[m] * c1 + B[m] * c2);
        }
    }
}

static void integrand_u(const orc_eval *E, const orc_out *o, double w, double wt, double *acc)
{
    const orc_lattice *L = E->L;
    double A[4], B[4];
    for (int c = 0; c < L->nc; ++c) {
        A[c] = vertex(L, E->x, c, o->b, o->dk, o->bk, o->w1 + w, w - o->w2p, o->u);
        B[c] = vertex(L, E->x, c, o->b, o->dk, o->bk, o->w1p + w, o->w2 - w, o->u);
    }
    if (L->nc == 2) {
        acc[0] += wt * (2.0 * A[0] * B[0] + A[0] * B[1] + A[1] * B[0]);
        acc[1] += wt * (3.0 * A[0] * B[0] + A[1] * B[1]);
    } else {
        acc[3] += wt * (A[3] * B[3] + A[0] * B[0] + A[1] * B[1] + A[2] * B[2]);
        acc[0] += wt * (A[3] * B[0] + A[0] * B[3] + A[1] * B[2] + A[2] * B[1]);
        acc[1] += wt * (A[3] * B[1] + A[1] * B[3] + A[2] * B[0] + A[0] * B[2]);
        acc[2] += wt * (A[3] * B[2] + A[2] * B[3] + A[0] * B[1] + A[1] * B[0]);
    }
}

/* ------------------------------------------- general (TRI) vertex ----- */

/*
 * TRI vertex (nc = 16): every basis function Gamma^{mu nu}, mu, nu = 0..3
 * (Sec. 3, Eq. 16), strain index 4 mu + nu.  Gamma^{mu nu} is real where
 * xi(mu) xi(nu) = 1 and imaginary where it is -1 (Eq. 18); the state holds
 * the real number r with Gamma = r, resp. Gamma = i r ("real
 * representation").  The channel products are formed literally: each
 * vertex becomes its spin tensor (Eq. 25), the spin sums of Eq. 24 run over
 * the 2x2x2x2 tensors, and the result is projected back on the basis with
 * Pauli traces.
 */
typedef double complex cplx;

static const cplx PAULI[4][2][2] = {
    {{1.0, 0.0}, {0.0, 1.0}},
    {{0.0, 1.0}, {1.0, 0.0}},
    {{0.0, -I}, {I, 0.0}},
    {{1.0, 0.0}, {0.0, -1.0}}};

static double xi_of(int m) { return m == 0 ? 1.0 : -1.0; }

/* The stored octant (s >= u >= 0, t >= 0) interpolated (Eq. 37) for all 16
 * strains; corners with s < u through the s <-> u relation (R4). */
static void gamma_octant(const orc_lattice *L, const double *x, int b1, int k,
                         double s, double t, double u, double g[4][4])
{
    int sa[2], ta[2], ua[2];
    double fs[2], ft[2], fu[2];
    bracket(L, s, &sa[0], &sa[1], &fs[0], &fs[1]);
    bracket(L, t, &ta[0], &ta[1], &ft[0], &ft[1]);
    bracket(L, u, &ua[0], &ua[1], &fu[0], &fu[1]);
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) g[m][n] = 0.0;
    for (int iu = 0; iu < 2; ++iu)
        for (int it = 0; it < 2; ++it)
            for (int is = 0; is < 2; ++is) {
                double wgt = fu[iu] * ft[it] * fs[is];
                if (wgt == 0.0) continue;
                int a = sa[is], c = ua[iu];
                for (int m = 0; m < 4; ++m)
                    for (int n = 0; n < 4; ++n) {
                        double v;
                        if (a >= c) v = x[vidx(L, 4 * m + n, b1, a, ta[it], c, k)];
                        else v = -xi_of(n) * x[vidx(L, 4 * m + n, b1, c, ta[it], a, k)];
                        g[m][n] += wgt * v;
                    }
            }
}

/* Gamma^{mu nu}_{i1 i2}(s,t,u) in the real representation between site
 * (b1, cell 0) and site (b2, cell d), through the relations of Eq. 18;
 * zero outside the truncation range (Eq. 34). */
static void gamma16(const orc_lattice *L, const double *x, int b1, const int d[3], int b2,
                    double s, double t, double u, double g[4][4])
{
    double h[4][4];
    const int nd[3] = {-d[0], -d[1], -d[2]};
    if (s < 0.0) {          /* Gamma^{mu nu}_{i1 i2}(s,t,u) = Gamma^{nu mu}_{i2 i1}(-s,t,u) */
        gamma16(L, x, b2, nd, b1, -s, t, u, h);
        for (int m = 0; m < 4; ++m)
            for (int n = 0; n < 4; ++n) g[m][n] = h[n][m];
        return;
    }
    if (t < 0.0) {          /* = xi(mu) xi(nu) Gamma^{mu nu}_{i1 i2}(s,-t,u) */
        gamma16(L, x, b1, d, b2, s, -t, u, h);
        for (int m = 0; m < 4; ++m)
            for (int n = 0; n < 4; ++n) g[m][n] = xi_of(m) * xi_of(n) * h[m][n];
        return;
    }
    if (u < 0.0) {          /* = xi(mu) xi(nu) Gamma^{nu mu}_{i2 i1}(s,t,-u) */
        gamma16(L, x, b2, nd, b1, s, t, -u, h);
        for (int m = 0; m < 4; ++m)
            for (int n = 0; n < 4; ++n) g[m][n] = xi_of(m) * xi_of(n) * h[n][m];
        return;
    }
    if (s < u) {            /* = -xi(nu) Gamma^{mu nu}_{i1 i2}(u,t,s) */
        gamma16(L, x, b1, d, b2, u, t, s, h);
        for (int m = 0; m < 4; ++m)
            for (int n = 0; n < 4; ++n) g[m][n] = -xi_of(n) * h[m][n];
        return;
    }
    int k = site_of(L, b1, d, b2);
    if (k < 0) {
        for (int m = 0; m < 4; ++m)
            for (int n = 0; n < 4; ++n) g[m][n] = 0.0;
        return;
    }
    gamma_octant(L, x, b1, k, s, t, u, g);
}

/* Spin tensor V[a'][b'][a][b] = sum Gamma^{mu nu} sigma^mu_{a'a} sigma^nu_{b'b} (Eq. 25). */
static void spin_tensor(const double g[4][4], cplx V[2][2][2][2])
{
    memset(V, 0, sizeof(cplx) * 16);
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            if (g[m][n] == 0.0) continue;
            cplx gv = xi_of(m) * xi_of(n) > 0.0 ? (cplx)g[m][n] : I * g[m][n];
            for (int p = 0; p < 2; ++p)
                for (int a = 0; a < 2; ++a) {
                    if (PAULI[m][p][a] == 0.0) continue;
                    for (int q = 0; q < 2; ++q)
                        for (int b = 0; b < 2; ++b)
                            V[p][q][a][b] += gv * PAULI[m][p][a] * PAULI[n][q][b];
                }
        }
}

static void spin_tensor_at(const orc_lattice *L, const double *x, int b1, const int d[3], int b2,
                           double s, double t, double u, cplx V[2][2][2][2])
{
    double g[4][4];
    gamma16(L, x, b1, d, b2, s, t, u, g);
    spin_tensor(g, V);
}

/* Basis functions of a spin tensor, Gamma^{mu nu} = (1/4) sum_{a'b'ab}
 * V[a'][b'][a][b] sigma^mu_{a a'} sigma^nu_{b b'}, added times wt to acc in
 * the real representation (real part where xi xi = 1, imaginary part where
 * it is -1; the other part vanishes by Eq. 18). */
static void project_add(cplx P[2][2][2][2], double wt, double *acc)
{
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            cplx v = 0.0;
            for (int p = 0; p < 2; ++p)
                for (int q = 0; q < 2; ++q)
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b)
                            v += P[p][q][a][b] * PAULI[m][a][p] * PAULI[n][b][q];
            v *= 0.25;
            acc[4 * m + n] += wt * (xi_of(m) * xi_of(n) > 0.0 ? creal(v) : cimag(v));
        }
}

/* s channel: legs (1',2';3,4) times (3,4;1,2), summed over the spins of 3, 4. */
static void integrand_s_tri(const orc_eval *E, const orc_out *o, double w, double wt, double *acc)
{
    const orc_lattice *L = E->L;
    cplx A[2][2][2][2], B[2][2][2][2], P[2][2][2][2];
    spin_tensor_at(L, E->x, o->b, o->dk, o->bk, o->s, o->w1p - w, w - o->w2p, A);
    spin_tensor_at(L, E->x, o->b, o->dk, o->bk, o->s, w - o->w1, w - o->w2, B);
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q)
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    cplx v = 0.0;
                    for (int c = 0; c < 2; ++c)
                        for (int d = 0; d < 2; ++d) v += A[p][q][c][d] * B[c][d][a][b];
                    P[p][q][a][b] = v;
                }
    project_add(P, wt, acc);
}

/* t channel: the particle-hole RPA term -sum_j Gamma_{i1 j} Gamma_{j i2}
 * (legs (1',4;1,3) times (3,2';4,2)) and the two vertex corrections with the
 * on-site vertices at i2 (legs (2',3;4,2)) and at i1 (legs (4,1';1,3)). */
static void integrand_t_tri(const orc_eval *E, const orc_out *o, double w, double wt, double *acc)
{
    const orc_lattice *L = E->L;
    const int zero[3] = {0, 0, 0};
    cplx A[2][2][2][2], B[2][2][2][2], O[2][2][2][2], P[2][2][2][2];
    memset(P, 0, sizeof(P));
    for (int j = 0; j < L->nsites[o->b]; ++j) {
        const int *cj = &L->cell[((long)o->b * L->ns + j) * 3];
        int bj = L->bas[(long)o->b * L->ns + j];
        int d2[3] = {o->dk[0] - cj[0], o->dk[1] - cj[1], o->dk[2] - cj[2]};
        if (site_of(L, bj, d2, o->bk) < 0) continue;
        spin_tensor_at(L, E->x, o->b, cj, bj, o->w1 + w, o->t, o->w1p - w, A);
        spin_tensor_at(L, E->x, bj, d2, o->bk, w + o->w2p, o->t, w - o->w2, B);
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q)
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 2; ++c)
                            for (int d = 0; d < 2; ++d) P[p][q][a][b] -= A[p][d][a][c] * B[c][q][d][b];
    }
    spin_tensor_at(L, E->x, o->b, o->dk, o->bk, o->w1 + w, o->t, o->w1p - w, A);
    spin_tensor_at(L, E->x, o->bk, zero, o->bk, o->w2p + w, o->w2 - w, -o->t, O);
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q)
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int c = 0; c < 2; ++c)
                        for (int d = 0; d < 2; ++d) P[p][q][a][b] += A[p][d][a][c] * O[q][c][d][b];
    spin_tensor_at(L, E->x, o->b, zero, o->b, o->w1 + w, w - o->w1p, -o->t, O);
    spin_tensor_at(L, E->x, o->b, o->dk, o->bk, w + o->w2p, o->t, w - o->w2, B);
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q)
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int c = 0; c < 2; ++c)
                        for (int d = 0; d < 2; ++d) P[p][q][a][b] += O[d][p][a][c] * B[c][q][d][b];
    project_add(P, wt, acc);
}

/* u channel: legs (4,2';1,3) times (1',3;4,2). */
static void integrand_u_tri(const orc_eval *E, const orc_out *o, double w, double wt, double *acc)
{
    const orc_lattice *L = E->L;
    cplx A[2][2][2][2], B[2][2][2][2], P[2][2][2][2];
    spin_tensor_at(L, E->x, o->b, o->dk, o->bk, o->w1 + w, w - o->w2p, o->u, A);
    spin_tensor_at(L, E->x, o->b, o->dk, o->bk, o->w1p + w, o->w2 - w, o->u, B);
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q)
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    cplx v = 0.0;
                    for (int c = 0; c < 2; ++c)
                        for (int d = 0; d < 2; ++d) v += A[d][q][a][c] * B[p][c][d][b];
                    P[p][q][a][b] = v;
                }
    project_add(P, wt, acc);
}

/* Eq. 23's spin sums for the TRI vertex at spin up (alpha_1 = 0):
 * sum_{a2} V_{0j}[0][a2][0][a2] over the sites j in range of basis site 0
 * at (w+x, 0, w-x), minus sum_{a2} V_{00}[a2][0][0][a2] at (w+x, x-w, 0). */
static double sigma_sum_tri(const orc_lattice *L, const double *x, double w, double xx)
{
    const int zero[3] = {0, 0, 0};
    cplx V[2][2][2][2];
    cplx f = 0.0;
    for (int k = 0; k < L->nsites[0]; ++k) {
        spin_tensor_at(L, x, 0, &L->cell[(long)k * 3], L->bas[k], w + xx, 0.0, w - xx, V);
        for (int a2 = 0; a2 < 2; ++a2) f += V[0][a2][0][a2];
    }
    spin_tensor_at(L, x, 0, zero, 0, w + xx, xx - w, 0.0, V);
    for (int a2 = 0; a2 < 2; ++a2) f -= V[a2][0][0][a2];
    return creal(f);
}

typedef void (*integrand_fn)(const orc_eval *, const orc_out *, double, double, double *);

/*
 * One channel: (1/2pi) * integral of the bubble times the channel integrand.
 * partner(w) = ps * w + pc  (s: pc - w; t: w - t; u: u + w) and its zero c.
 */
static void channel(const orc_eval *E, const orc_out *o, integrand_fn fn,
                    double ps, double pc, double *acc)
{
    const orc_lattice *L = E->L;
    double lam = E->lam;
    double loc[MAXC] = {0.0};

    /* delta parts (R1): the S in Skat(partner) and the S in Skat(w) */
    for (int sx = 0; sx < 2; ++sx) {
        double xx = sx == 0 ? lam : -lam;
        double st = 1.0 / (xx - sig_at(E, xx));
        double winv = (xx - pc) / ps;        /* partner(winv) == xx */
        double pxx = ps * xx + pc;           /* partner of w == xx */
        double g1 = theta_half(winv, lam);     /* the propagator vanishes where theta does */
        double g2 = theta_half(pxx, lam);
        if (g1 != 0.0) g1 *= gbare(E, winv);
        if (g2 != 0.0) g2 *= gbare(E, pxx);
        if (g1 != 0.0) fn(E, o, winv, -st * g1, loc);
        if (g2 != 0.0) fn(E, o, xx, -st * g2, loc);
    }

    /* Katanin part (R2): trapezoid over the pieces of the domain */
    double c = -pc / ps;
    double lo[MAXPIECE], hi[MAXPIECE];
    int np = pieces(c, lam, L->w[L->nf - 1], lo, hi);
    double *nodes = (double *)malloc(sizeof(double) * (2 * L->nf + 4));
    for (int ip = 0; ip < np; ++ip) {
        int nn = piece_nodes(L, lo[ip], hi[ip], nodes);
        for (int i = 0; i < nn; ++i) {
            double wl = i > 0 ? 0.5 * (nodes[i] - nodes[i - 1]) : 0.0;
            double wr = i + 1 < nn ? 0.5 * (nodes[i + 1] - nodes[i]) : 0.0;
            double w = nodes[i];
            double p = ps * w + pc;
            double gw = gbare(E, w), gp = gbare(E, p);
            double kat = gw * gp * gp * dsig_at(E, p) + gp * gw * gw * dsig_at(E, w);
            fn(E, o, w, (wl + wr) * kat, loc);
        }
    }
    free(nodes);
    for (int c = 0; c < L->nc; ++c) acc[c] += loc[c] / TWO_PI;
}

/*
 * Flow of the vertex element (basis b, listed site k) at mesh indices
 * s = w[a], t = w[it], u = w[c] with a >= c.  `dsig` must hold the
 * self-energy flow of the same state at the same Lambda (Katanin term).
 */
void orc_vertex_rhs_element(const orc_lattice *L, double lam, const double *x, const double *dsig,
                            int b, int k, int a, int it, int c, double *out)
{
    orc_eval E = {L, x, dsig, lam};
    orc_out o;
    o.b = b; o.k = k;
    o.bk = L->bas[(long)b * L->ns + k];
    for (int i = 0; i < 3; ++i) o.dk[i] = L->cell[((long)b * L->ns + k) * 3 + i];
    o.s = L->w[a]; o.t = L->w[it]; o.u = L->w[c];
    /* s = w1'+w2', t = w1'-w1, u = w1'-w2 and w1'+w2' = w1+w2 (Eq. 17) */
    o.w1p = 0.5 * (o.s + o.t + o.u);
    o.w2p = 0.5 * (o.s - o.t - o.u);
    o.w1 = 0.5 * (o.s - o.t + o.u);
    o.w2 = 0.5 * (o.s + o.t - o.u);
    double acc[MAXC] = {0.0};
    const int tri = L->nc == 16;
    channel(&E, &o, tri ? integrand_s_tri : integrand_s, -1.0, o.s, acc);   /* partner s - w */
    channel(&E, &o, tri ? integrand_t_tri : integrand_t, 1.0, -o.t, acc);   /* partner w - t */
    channel(&E, &o, tri ? integrand_u_tri : integrand_u, 1.0, o.u, acc);    /* partner u + w */
    for (int comp = 0; comp < L->nc; ++comp) out[comp] = acc[comp];
}

/* Full right-hand side: sigma flow, then every vertex element. */
void orc_rhs(const orc_lattice *L, double lam, const double *x, double *dx, int nthreads)
{
    double *dsig = dx;   /* the sigma part of the output doubles as dsig */
    orc_sigma_rhs(L, lam, x, dsig);
    long nsu = n_su(L);
    long total = (long)L->nb * nsu * L->nf;
    memset(dx + L->nf, 0, sizeof(double) * (size_t)(orc_state_size(L) - L->nf));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (long q = 0; q < total; ++q) {
        int b = (int)(q / (nsu * L->nf));
        long r = q % (nsu * L->nf);
        int su = (int)(r / L->nf), it = (int)(r % L->nf);
        int a = 0;
        while (su_index(a + 1, 0) <= su) ++a;
        int c = su - (int)su_index(a, 0);
        for (int k = 0; k < L->nsites[b]; ++k) {
            double out[MAXC];
            orc_vertex_rhs_element(L, lam, x, dsig, b, k, a, it, c, out);
            for (int comp = 0; comp < L->nc; ++comp) dx[vidx(L, comp, b, a, it, c, k)] = out[comp];
        }
    }
}

/*
 * Every vertex element of a list of frequency triples (all basis sites and
 * listed sites), written to out[q][b][k][nc].  Used for sampled comparisons
 * and for the CPU baseline timing.
 */
void orc_vertex_rhs_triples(const orc_lattice *L, double lam, const double *x, const double *dsig,
                            int nq, const int *a_list, const int *t_list, const int *c_list,
                            double *out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
#endif
    for (int q = 0; q < nq; ++q)
        for (int b = 0; b < L->nb; ++b)
            for (int k = 0; k < L->nsites[b]; ++k)
                orc_vertex_rhs_element(L, lam, x, dsig, b, k, a_list[q], t_list[q], c_list[q],
                                       &out[(((long)q * L->nb + b) * L->ns + k) * L->nc]);
}

/* ------------------------------------------------------- correlations -- */

/*
 * Two-spin correlations (Eq. 30 contracted with Eq. 25, R5), one per strain:
 *   chi^m_ij = d_ij (1/4pi) I g^2 - (1/16pi^2) II g1^2 g2^2
 *              [4 G^m_ij(w1+w2, 0, w1-w2) + d_ij X^m(w1+w2, w2-w1, 0)]
 * with g = 1/(w - sig(w)) on |w| >= Lambda (G^2 = -g^2) and the on-site
 * exchange term
 *   SU(2): X^zz = 2 Gs_ii - 2 Gd_ii,  X^00 = -(6 Gs_ii + 2 Gd_ii);
 *   XYZ:   X^m = -2 sum_n e(m,n) G^n_ii (e as in the t channel).
 * out[m][b][k] for every strain m (SU(2): zz, 00; XYZ: xx, yy, zz, 00).
 */
void orc_chi_comps(const orc_lattice *L, double lam, const double *x, double *out)
{
    orc_eval E = {L, x, NULL, lam};
    double wmax = L->w[L->nf - 1];
    int cap = 2 * (2 * L->nf + 4);
    double *nw = (double *)malloc(sizeof(double) * cap);
    double *ww = (double *)malloc(sizeof(double) * cap);
    double *g2 = (double *)malloc(sizeof(double) * cap);
    double *tmp = (double *)malloc(sizeof(double) * (2 * L->nf + 4));
    int n = 0;
    double lo[2] = {-wmax, lam}, hi[2] = {-lam, wmax};
    for (int ip = 0; ip < 2; ++ip) {
        if (!(lo[ip] < hi[ip])) continue;
        int nn = piece_nodes(L, lo[ip], hi[ip], tmp);
        for (int i = 0; i < nn; ++i) {
            double wl = i > 0 ? 0.5 * (tmp[i] - tmp[i - 1]) : 0.0;
            double wr = i + 1 < nn ? 0.5 * (tmp[i + 1] - tmp[i]) : 0.0;
            nw[n] = tmp[i];
            ww[n] = wl + wr;
            double g = gbare(&E, tmp[i]);
            g2[n] = g * g;
            ++n;
        }
    }
    double bubble = 0.0;
    for (int i = 0; i < n; ++i) bubble += ww[i] * g2[i];
    bubble /= 2.0 * TWO_PI;
    const double pref = 1.0 / (4.0 * TWO_PI * TWO_PI);   /* 1/(16 pi^2) */
    const int zero[3] = {0, 0, 0};
    const int nc = L->nc;
    const long plane = (long)L->nb * L->ns;
    for (int b = 0; b < L->nb; ++b)
        for (int k = 0; k < L->nsites[b]; ++k) {
            const int *ck = &L->cell[((long)b * L->ns + k) * 3];
            int bk = L->bas[(long)b * L->ns + k];
            int onsite = (k == 0);
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    double w1 = nw[i], w2 = nw[j];
                    double f = ww[i] * ww[j] * g2[i] * g2[j];
                    double t[4] = {0.0, 0.0, 0.0, 0.0}, e[4] = {0.0, 0.0, 0.0, 0.0};
                    for (int m = 0; m < nc; ++m) t[m] = 4.0 * vertex(L, x, m, b, ck, bk, w1 + w2, 0.0, w1 - w2);
                    if (onsite) {
                        for (int m = 0; m < nc; ++m) e[m] = vertex(L, x, m, b, zero, b, w1 + w2, w2 - w1, 0.0);
                        if (nc == 2) {
                            t[0] += 2.0 * e[0] - 2.0 * e[1];
                            t[1] -= 6.0 * e[0] + 2.0 * e[1];
                        } else {
                            for (int m = 0; m < 4; ++m) {
                                double xm = 0.0;
                                for (int q = 0; q < 4; ++q) xm += xyz_sign(m, q) * e[q];
                                t[m] += -2.0 * xm;
                            }
                        }
                    }
                    for (int m = 0; m < nc; ++m) acc[m] += f * t[m];
                }
            for (int m = 0; m < nc; ++m) {
                double v = -pref * acc[m];
                if (onsite) v += bubble;
                out[m * plane + (long)b * L->ns + k] = v;
            }
        }
    free(nw); free(ww); free(g2); free(tmp);
}

/* SU(2): chi^{zz} and chi^{00} of every (basis, site) element (orc_chi_comps). */
void orc_chi(const orc_lattice *L, double lam, const double *x, double *chi_zz, double *chi_dd)
{
    const long plane = (long)L->nb * L->ns;
    double *both = (double *)malloc(sizeof(double) * 2 * plane);
    orc_chi_comps(L, lam, x, both);
    memcpy(chi_zz, both, sizeof(double) * plane);
    memcpy(chi_dd, both + plane, sizeof(double) * plane);
    free(both);
}

/*
 * TRI correlations chi^{mu nu}_ij for mu, nu = 0..3 (Eq. 30, R5) from the
 * spin tensors: with G = -i g on |w| >= Lambda,
 *   chi^{mu nu}_ij = d_ij d_{mu nu} (1/4pi) I g^2
 *       - (1/16pi^2) II g1^2 g2^2 sum sigma^mu_{a1 a1'} sigma^nu_{a2 a2'}
 *         [V_ij(w1+w2, 0, w1-w2) - d_ij V^x_ii(w1+w2, w2-w1, 0)][a1'][a2'][a1][a2]
 * where V^x is the on-site spin tensor with its two outgoing legs exchanged
 * (the -(1' <-> 2') part of Eq. 16).  out_re / out_im [16][nb][ns], index
 * 4 mu + nu first.
 */
void orc_chi_tri(const orc_lattice *L, double lam, const double *x, double *out_re, double *out_im)
{
    orc_eval E = {L, x, NULL, lam};
    double wmax = L->w[L->nf - 1];
    int cap = 2 * (2 * L->nf + 4);
    double *nw = (double *)malloc(sizeof(double) * cap);
    double *ww = (double *)malloc(sizeof(double) * cap);
    double *g2 = (double *)malloc(sizeof(double) * cap);
    double *tmp = (double *)malloc(sizeof(double) * (2 * L->nf + 4));
    int n = 0;
    double lo[2] = {-wmax, lam}, hi[2] = {-lam, wmax};
    for (int ip = 0; ip < 2; ++ip) {
        if (!(lo[ip] < hi[ip])) continue;
        int nn = piece_nodes(L, lo[ip], hi[ip], tmp);
        for (int i = 0; i < nn; ++i) {
            double wl = i > 0 ? 0.5 * (tmp[i] - tmp[i - 1]) : 0.0;
            double wr = i + 1 < nn ? 0.5 * (tmp[i + 1] - tmp[i]) : 0.0;
            nw[n] = tmp[i];
            ww[n] = wl + wr;
            double g = gbare(&E, tmp[i]);
            g2[n] = g * g;
            ++n;
        }
    }
    double bubble = 0.0;
    for (int i = 0; i < n; ++i) bubble += ww[i] * g2[i];
    bubble /= 2.0 * TWO_PI;
    const double pref = 1.0 / (4.0 * TWO_PI * TWO_PI);   /* 1/(16 pi^2) */
    const int zero[3] = {0, 0, 0};
    const long plane = (long)L->nb * L->ns;
    for (int b = 0; b < L->nb; ++b)
        for (int k = 0; k < L->nsites[b]; ++k) {
            const int *ck = &L->cell[((long)b * L->ns + k) * 3];
            int bk = L->bas[(long)b * L->ns + k];
            int onsite = (k == 0);
            cplx acc[16];
            for (int c = 0; c < 16; ++c) acc[c] = 0.0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    double w1 = nw[i], w2 = nw[j];
                    double f = ww[i] * ww[j] * g2[i] * g2[j];
                    cplx V[2][2][2][2], X[2][2][2][2];
                    spin_tensor_at(L, x, b, ck, bk, w1 + w2, 0.0, w1 - w2, V);
                    if (onsite) {
                        spin_tensor_at(L, x, b, zero, b, w1 + w2, w2 - w1, 0.0, X);
                        for (int p = 0; p < 2; ++p)
                            for (int q = 0; q < 2; ++q)
                                for (int a = 0; a < 2; ++a)
                                    for (int c = 0; c < 2; ++c) V[p][q][a][c] -= X[q][p][a][c];
                    }
                    for (int m = 0; m < 4; ++m)
                        for (int nn = 0; nn < 4; ++nn) {
                            cplx v = 0.0;
                            for (int a1 = 0; a1 < 2; ++a1)
                                for (int a1p = 0; a1p < 2; ++a1p) {
                                    if (PAULI[m][a1][a1p] == 0.0) continue;
                                    for (int a2 = 0; a2 < 2; ++a2)
                                        for (int a2p = 0; a2p < 2; ++a2p)
                                            v += PAULI[m][a1][a1p] * PAULI[nn][a2][a2p] * V[a1p][a2p][a1][a2];
                                }
                            acc[4 * m + nn] += f * v;
                        }
                }
            for (int c = 0; c < 16; ++c) {
                cplx v = -pref * acc[c];
                if (onsite && c % 5 == 0) v += bubble;   /* mu == nu */
                out_re[c * plane + (long)b * L->ns + k] = creal(v);
                out_im[c * plane + (long)b * L->ns + k] = cimag(v);
            }
        }
    free(nw); free(ww); free(g2); free(tmp);
}
