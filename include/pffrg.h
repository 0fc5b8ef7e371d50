/*
 * pffrg.h -- C ABI of the MI355X pf-FRG flow library (libpffrg.so).
 *
 * The library computes the SU(2) pseudofermion functional-renormalization-
 * group flow of arXiv:2109.13317: the right-hand side of the self-energy and
 * two-particle-vertex flow equations at cutoff Lambda (Sec. 3, Eq. 23 and
 * Eq. 24 with the Katanin propagator of Eq. 13), explicit Runge-Kutta
 * integration in Lambda (Sec. 4.3), and the two-spin correlations chi_ij and
 * chi(k) (Eq. 30, Eq. 31).  All arithmetic runs in HIP kernels on the GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers named d_* are device pointers to memory the caller owns (for
 * example a torch tensor's data_ptr()).  The library never frees them and
 * never keeps them after the call returns.  Host arrays passed to
 * pffrg_create are copied; the caller may free them afterwards.
 *
 * Every call returns a pffrg_status.  On failure a message is available
 * from pffrg_last_error() (thread-local, valid until the next call on the
 * same thread).  No C++ exception crosses this boundary.
 *
 * Work is enqueued on the context's stream (a hipStream_t, passed here as
 * void*; NULL means the default stream) and is asynchronous unless stated.
 * All device memory a context needs is allocated in pffrg_create; no later
 * call allocates.
 *
 * Flow state layout (FP64, n_freq = Nw, n_pairs = Ns):
 *   state[0 .. Nw)              sig(w_n) = Im Sigma(w_n) on the positive mesh
 *                               (Sigma is purely imaginary and odd, Eq. 15)
 *   state[Nw + V*0 .. )         spin vertex   Gs = Gamma^{33} (= 11 = 22)
 *   state[Nw + V*1 .. )         density vertex Gd = Gamma^{00}
 * with V = T*Ns and T = Nw*Nw*(Nw+1)/2.  Inside each strain the index of
 * (s = w_a, t = w_t, u = w_c), a >= c, pair p is
 *   ((a*(a+1)/2 + c) * Nw + t) * Ns + p,
 * i.e. the (s,u) wedge outermost, then t, then the pair (the memory layout
 * of Sec. 4.4 for the two SU(2) strains).  Values at other frequencies
 * follow from the symmetry relations (Eq. 18) and trilinear interpolation
 * with constant extrapolation (Eq. 37).
 */
#ifndef PFFRG_H
#define PFFRG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PFFRG_OK = 0,
    PFFRG_EINVAL = -1,        /* bad table, mesh, size, pointer or Lambda <= 0 */
    PFFRG_EHIP = -2,          /* HIP runtime failure */
    PFFRG_ENOMEM = -3,        /* device allocation failed in pffrg_create */
    PFFRG_EDIVERGED = -4,     /* NaN/Inf in the state, or step size below hmin */
    PFFRG_EUNSUPPORTED = -5   /* option or size beyond what the library supports */
} pffrg_status;

typedef enum {
    PFFRG_FP64 = 0,           /* every kernel in FP64 */
    PFFRG_FP32 = 1            /* vertex quadrature and lattice sums in FP32 with
                                 compensated accumulation; state, propagators,
                                 self-energy flow, steps and chi in FP64 */
} pffrg_precision;

typedef struct pffrg_ctx pffrg_ctx;

/*
 * Symmetry-reduced lattice (Sec. 4.1).  The reference site is basis site 0;
 * pair p stands for the orbit of site j_p under the point group fixing the
 * reference site, truncated at bond distance L (Eq. 34).  Pair 0 must be the
 * on-site pair.
 *   swap[p]      pair of (j_p, i_ref), i.e. Gamma_{j i} for Gamma_{i j}
 *   mult[p]      number of sites in the orbit of pair p (>= 1)
 *   rpa_*        tabulated lattice sums: for output pair p, the terms
 *                rpa_off[p] <= q < rpa_off[p+1] contribute
 *                rpa_cnt[q] * Gamma_{rpa_ka[q]} * Gamma_{rpa_kb[q]} to
 *                sum_j Gamma_{i_ref j} Gamma_{j j_p}
 *   coupling[p]  Heisenberg coupling J of the bond (i_ref, j_p), 0 if none;
 *                each unordered bond counted once (Eq. 21: Gs = J/4); finite
 *   n_basis, n_sites_total, site_pair[b*n_sites_total + k], site_pos[..*3]
 *                for every basis site b the sites within range of b, their
 *                reduced pair (-1 pads short lists; values below -1 are
 *                rejected) and Cartesian position;
 *   basis_pos    [n_basis*3] Cartesian basis-site positions (chi(k))
 */
typedef struct {
    int n_pairs;
    const int *swap;
    const int *mult;
    const int *rpa_off;
    const int *rpa_ka;
    const int *rpa_kb;
    const int *rpa_cnt;
    const double *coupling;
    int n_basis;
    int n_sites_total;
    const int *site_pair;
    const double *site_pos;
    const double *basis_pos;
} pffrg_lattice;

/* Positive frequency mesh, strictly ascending, n_freq >= 2, omega[0] > 0
 * (Sec. 4.2; negative frequencies are implied by symmetry). */
typedef struct {
    int n_freq;
    const double *omega;
} pffrg_mesh;

/* ---------------------------------------------------------- lifecycle -- */

/* Copy the tables to the device and allocate every buffer the context will
 * use.  `stream` is a hipStream_t or NULL.  The mesh and every table are
 * checked on the host before the first HIP call: a null or malformed one
 * (an index out of range, rpa_off descending, a count outside [1, 32767], a
 * non-positive, non-finite or unsorted frequency, a non-finite coupling, an
 * unknown precision) gives PFFRG_EINVAL, more than 128 frequencies or pairs
 * beyond the kernel build PFFRG_EUNSUPPORTED, with *out left NULL and
 * nothing allocated; a failed device allocation gives PFFRG_ENOMEM. */
pffrg_status pffrg_create(const pffrg_lattice *lat, const pffrg_mesh *mesh,
                          pffrg_precision prec, void *stream, pffrg_ctx **out);

/* An XYZ context (Sec. 2: H = sum over bonds of Jx S^x S^x + Jy S^y S^y +
 * Jz S^z S^z; Sec. 3: only the diagonal vertex components flow).
 * coupling3[m * n_pairs + p] (host, copied) is J^m of the bond (i_ref, j_p)
 * for m = x, y, z; lat->coupling is not read (it may be NULL).  The pair
 * tables must reduce by symmetries that map every bond to one with equal
 * (Jx, Jy, Jz).  The state then holds four strains,
 *   sig | Gx | Gy | Gz | Gd   (V = T*Ns elements each, the layout above),
 * Gx, Gy, Gz even under s <-> u like the SU(2) spin strain, Gd odd; the
 * initial condition is G^m = J^m/4, Gd = 0; pffrg_chi returns [4][Ns]
 * (chi^xx, chi^yy, chi^zz, chi^00) and pffrg_chi_k sums chi^xx + chi^yy +
 * chi^zz (Eq. 31).  Up to 32 pairs, as for SU(2).  PFFRG_FP32 runs the
 * vertex interpolation, channel products and lattice-sum matrices in FP32
 * with compensated chunk sums (the self-energy, tables, contraction, state
 * and chi stay FP64), as for SU(2); the reverse-mode calls
 * (pffrg_init_state_from, pffrg_*_vjp) give PFFRG_EUNSUPPORTED on an XYZ
 * context.  NULL coupling3 or a non-finite coupling: PFFRG_EINVAL. */
pffrg_status pffrg_create_xyz(const pffrg_lattice *lat, const double *coupling3, const pffrg_mesh *mesh,
                              pffrg_precision prec, void *stream, pffrg_ctx **out);

/* Spin transformations of a TRI context's pair tables (Sec. 4.1: lattice
 * symmetries joined with a global permutation of the spin components).  A
 * rotation W is a signed permutation matrix with det W = +1 (the sign that
 * makes a permutation a rotation of the spin axes), given by its rows: row a
 * holds sign(v) in column |v| - 1, v = rot[3 r + a] in {+-1, +-2, +-3}.  A pair
 * reached through a rotation holds W Gamma W^T on its spin indices (the
 * density index untouched).  All arrays are host pointers, copied. */
typedef struct {
    int n_rot;              /* rotations, 1..24; rotation 0 must be the identity */
    const int *rot;         /* [n_rot][3] rows as above */
    const int *swap_rot;    /* [n_pairs]: Gamma_{j_p i_ref} = W Gamma_{swap[p]} W^T */
    const int *rpa_rot_a;   /* [n_terms] (rpa_off order): Gamma_{i_ref k} = W Gamma_{ka} W^T */
    const int *rpa_rot_b;   /* [n_terms]: Gamma_{k j_p} = W Gamma_{kb} W^T */
    const int *site_rot;    /* [n_basis][n_sites_total]: rotation of each site's pair (site_pair) */
} pffrg_spin_rot;

/* A TRI context: the general time-reversal invariant model (Sec. 2:
 * H = sum J_ij^{mu nu} S_i^mu S_j^nu with real 3x3 matrices; Sec. 3: all
 * sixteen vertex components Gamma^{mu nu}, Eq. 16, with the symmetries of
 * Eq. 18).  coupling9[9 p + 3 a + b] (host, copied) is M^{ab} of the bond
 * (i_ref, j_p) in the term S_ref . M . S_j, a, b = x, y, z; lat->coupling is
 * not read (it may be NULL).  The pair tables must reduce by lattice
 * symmetries that map every directed bond to one with the same matrix (no
 * spin rotation or permutation).  The state holds sixteen strains,
 *   sig | G^{00} | G^{01} | ... | G^{33}   (strain 4 mu + nu, V = T*Ns each),
 * index 0 the density, 1..3 x, y, z; G^{mu nu} is Gamma^{mu nu} where
 * xi(mu) xi(nu) = 1 and its imaginary part where it is -1 (those components
 * are imaginary, Eq. 18).  Initial condition G^{ab} = M^{ab}/4 for
 * a, b = x, y, z, the rest 0 (Eq. 22).  The self-energy flow takes the spin
 * average of the sums of Eq. 23 (it keeps Sigma imaginary).  pffrg_chi returns
 * [16][Ns], the real parts of chi^{mu nu} at 4 mu + nu (Eq. 30); pffrg_chi_k
 * sums chi^{xx} + chi^{yy} + chi^{zz} (Eq. 31); pffrg_chi_sites spreads all
 * sixteen.  srot (may be NULL: pure lattice symmetries) carries the spin
 * rotations of tables reduced by joint lattice and spin transformations
 * (Sec. 4.1); the kernels then apply them on every exchanged pair, lattice-sum
 * factor and chi site.  Up to 64 pairs, FP64 only (PFFRG_FP32:
 * PFFRG_EUNSUPPORTED); the reverse-mode calls give PFFRG_EUNSUPPORTED on a TRI
 * context.  NULL coupling9, a non-finite coupling, or a rotation table that is
 * not as above (ids out of range, rotation 0 not the identity, a row that is
 * not a signed unit vector, det W != +1): PFFRG_EINVAL. */
pffrg_status pffrg_create_tri(const pffrg_lattice *lat, const double *coupling9, const pffrg_spin_rot *srot,
                              const pffrg_mesh *mesh, pffrg_precision prec, void *stream, pffrg_ctx **out);
pffrg_status pffrg_destroy(pffrg_ctx *ctx);
pffrg_status pffrg_set_stream(pffrg_ctx *ctx, void *stream);

/* Number of doubles in one flow state (layout above). */
pffrg_status pffrg_state_size(const pffrg_ctx *ctx, size_t *n_doubles);

/* Initial condition at infinite cutoff (Eq. 14, Eq. 21): sig = 0,
 * Gs = coupling/4 for every frequency, Gd = 0. */
pffrg_status pffrg_init_state(pffrg_ctx *ctx, double *d_state);

/* ---------------------------------------------------------- the flow --- */

/* d_dstate = d state / d Lambda at cutoff `lambda` > 0: the self-energy flow
 * (Eq. 23) first, then the vertex flow (Eq. 24) whose Katanin term uses it.
 * d_state and d_dstate must not overlap. */
pffrg_status pffrg_rhs(pffrg_ctx *ctx, double lambda, const double *d_state, double *d_dstate);

/* Self-energy part only: d_dsig[Nw] = d sig/d Lambda (Eq. 23). */
pffrg_status pffrg_sigma_rhs(pffrg_ctx *ctx, double lambda, const double *d_state, double *d_dsig);

/* One explicit step from lam0 to lam1 (lam1 < lam0 for a downward flow),
 * updating d_state in place.  PFFRG_EULER is the paper's scheme (Eq. 42);
 * PFFRG_RK4 is the classical fourth-order Runge-Kutta step in Lambda with
 * stages at lam0, lam0 + h/2, lam0 + h/2, lam1 (h = lam1 - lam0). */
typedef enum { PFFRG_EULER = 0, PFFRG_RK4 = 1, PFFRG_DOPRI54 = 2 } pffrg_scheme;
pffrg_status pffrg_step(pffrg_ctx *ctx, pffrg_scheme scheme, double lam0, double lam1, double *d_state);

/* Observer called after every accepted step with the new cutoff and device
 * pointers to chi per pair ([2][Ns]: zz then density) and chi(k) (or NULL
 * when no k-points were given).  It runs on the host after the stream has
 * been synchronised; a non-zero return stops the flow with PFFRG_OK. */
typedef int (*pffrg_observer)(double lambda, const double *d_chi_pairs, const double *d_chi_k,
                              void *user);

typedef struct {
    pffrg_scheme scheme;
    /* fixed-step schedules (EULER, RK4): the cutoff values, first = start */
    int n_lambda;
    const double *lambdas;      /* host array */
    /* adaptive (DOPRI54): Dormand-Prince 5(4) in l = ln Lambda from
     * lam_start down to lam_stop with mixed tolerance atol + rtol*|x| in the
     * max norm, first step h0 (in l, > 0), minimal step hmin */
    double lam_start, lam_stop, rtol, atol, h0, hmin;
    int max_steps;
    /* measurements after each accepted step: chi per pair always when an
     * observer is given; chi(k) at n_k points d_k[3*n_k] (device) if n_k > 0 */
    int n_k;
    const double *d_k;
    double *d_chi_k;            /* device output [n_k], passed to the observer */
    /* adaptive: resume != 0 continues an earlier flow from the position
     * (ln Lambda, step-ladder index) that pffrg_flow_position reported at one
     * of its accepted steps, with d_state the state accepted there; lam_start
     * is then ignored.  With the same mesh, lattice, precision, tolerances,
     * h0 and lam_stop the continued flow takes exactly the steps the earlier
     * one took after that point (bitwise the same states); with a lower
     * lam_stop it extends a finished flow. */
    int resume;
    int resume_ladder;
    double resume_log_lambda;
} pffrg_flow_opts;

/* Integrate d_state along the options' schedule.  Returns PFFRG_EDIVERGED
 * (with d_state holding the last finite state) if the state stops being
 * finite or the adaptive step falls below hmin.  The number of accepted
 * steps is written to *n_steps if it is not NULL. */
pffrg_status pffrg_flow(pffrg_ctx *ctx, const pffrg_flow_opts *opts, double *d_state,
                        pffrg_observer cb, void *user, int *n_steps);

/* Position of the last accepted step of the running (when called from the
 * observer) or last flow on this context: its cutoff, ln of it as the
 * integrator holds it, and the step-ladder index the adaptive controller
 * would start the next step from (fixed schedules: the index of the accepted
 * cutoff in the schedule).  These, with the state, are what a checkpoint
 * needs to resume the flow exactly (the paper's checkpoint files, Sec. 5.1).
 * Before any accepted step: PFFRG_EINVAL. */
pffrg_status pffrg_flow_position(pffrg_ctx *ctx, double *lambda, double *log_lambda, int *ladder);

/* --------------------------------------------------------- observables - */

/* Two-spin correlations per reduced pair at cutoff lambda (Eq. 30):
 * d_chi[0*Ns + p] = chi^{zz}_{i_ref j_p}, d_chi[1*Ns + p] = chi^{00}. */
pffrg_status pffrg_chi(pffrg_ctx *ctx, double lambda, const double *d_state, double *d_chi);

/* Structure factor (Eq. 31) per unit cell from chi per pair:
 * d_chi_k[q] = (1/n_basis) sum_b sum_j cos(k_q . (r_b - r_j)) 3 chi^{zz}_{b j}
 * for the n_k points d_k[3*q .. 3*q+2]. */
pffrg_status pffrg_chi_k(pffrg_ctx *ctx, const double *d_chi, int n_k, const double *d_k,
                         double *d_chi_k);

/* The correlations per reduced pair (d_chi as pffrg_chi returns them:
 * [strains][Ns], two strains for SU(2), four for XYZ) in the layout of the
 * paper's observable files (Sec. 5, output data: per basis site b of the
 * unit cell and per site k within range of it):
 * d_chi_sites[(m * n_basis + b) * n_sites_total + k] = d_chi[m * Ns +
 * site_pair[b * n_sites_total + k]], NaN where site_pair is -1 (a basis site
 * with fewer sites in range).  Both device arrays are the caller's;
 * d_chi_sites holds strains * n_basis * n_sites_total doubles.  NULL
 * pointers: PFFRG_EINVAL. */
pffrg_status pffrg_chi_sites(pffrg_ctx *ctx, const double *d_chi, double *d_chi_sites);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * correlations as pffrg_chi, d_chi[0*Ns + p] = chi^{zz}, d_chi[1*Ns + p] =
 * chi^{00}, with no context and no allocation.  The caller passes the mesh
 * d_omega[n_freq] (device, positive, strictly ascending, as for
 * pffrg_create), the pair exchange table d_swap[n_pairs] (device, entries in
 * [0, n_pairs), as pffrg_lattice.swap), the state (layout above) and the
 * output; work is enqueued on `stream` (a hipStream_t of the current device,
 * or NULL).  Device inputs are not read on the host, so their contents are
 * not checked.  The kernels' scratch (node lists and partial integrals,
 * PFFRG_NOALLOC_SCRATCH_BYTES) is a fixed device array that each device holds
 * until the process ends; its address is looked up on the first call with a
 * device current.  All calls on one device share it: calls that overlap on
 * one device race and must be ordered by the caller.  More than
 * PFFRG_NOALLOC_MAX_FREQ frequencies or PFFRG_NOALLOC_MAX_PAIRS pairs give
 * PFFRG_EUNSUPPORTED; a null pointer, n_freq < 2, n_pairs < 1 or a lambda
 * that is not finite and > 0 give PFFRG_EINVAL.  Asynchronous. */
#define PFFRG_NOALLOC_MAX_FREQ 128
#define PFFRG_NOALLOC_MAX_PAIRS 32
#define PFFRG_NOALLOC_SCRATCH_BYTES 14448
pffrg_status pffrg_chi_noalloc(int n_freq, const double *d_omega, int n_pairs, const int *d_swap, double lambda,
                               const double *d_state, double *d_chi, void *stream);

/* -------------------------------------------------------- reverse mode - */

/*
 * Gradients of observables with respect to the couplings through the whole
 * flow (reverse mode; FP64 whatever the context's precision).  The flow
 * equations (Eq. 23, Eq. 24) are differentiated as discretised: the same
 * mesh, interpolation, quadrature nodes and RK4 stages, so the results are
 * the exact derivatives of the computed chi up to rounding.
 */

/* Initial condition (as pffrg_init_state) for the couplings d_coupling[Ns]
 * (device) instead of the ones given at create. */
pffrg_status pffrg_init_state_from(pffrg_ctx *ctx, const double *d_coupling, double *d_state);

/* d_cot_state = J^T d_cot_dstate, J = d(pffrg_rhs output)/d(state) at
 * (lambda, d_state); all three arrays in the state layout, d_cot_state
 * overwritten and not overlapping the inputs. */
pffrg_status pffrg_rhs_vjp(pffrg_ctx *ctx, double lambda, const double *d_state, const double *d_cot_dstate,
                           double *d_cot_state);

/* d_cot_state = (d chi / d state)^T d_cot_chi for chi per pair (Eq. 30) at
 * (lambda, d_state); d_cot_chi as pffrg_chi's output ([2][Ns]). */
pffrg_status pffrg_chi_vjp(pffrg_ctx *ctx, double lambda, const double *d_state, const double *d_cot_chi,
                           double *d_cot_state);

/* d_cot_chi[2*Ns] = (d chi(k) / d chi)^T d_cot_chi_k for the structure
 * factor of pffrg_chi_k (Eq. 31) at the n_k points d_k. */
pffrg_status pffrg_chi_k_vjp(pffrg_ctx *ctx, const double *d_cot_chi_k, int n_k, const double *d_k,
                             double *d_cot_chi);

/* RK4 along lambdas (as pffrg_step per interval), storing the state at the
 * start of every step: d_checkpoints[(n_lambda-1) * state size] (device,
 * caller-owned; 120 steps of the honeycomb range-6 workload take 454 MB).
 * PFFRG_EDIVERGED if the final state is not finite. */
pffrg_status pffrg_flow_checkpoints(pffrg_ctx *ctx, int n_lambda, const double *lambdas, double *d_state,
                                    double *d_checkpoints);

/* Discrete adjoint of that flow: on entry d_cot holds the cotangent of the
 * final state, on return that of the initial state (each step's stages are
 * recomputed from its checkpoint and transposed).  If d_dcoupling[Ns] is not
 * NULL it receives the gradient with respect to the couplings of the
 * initial condition (Gs = coupling / 4, Eq. 21). */
pffrg_status pffrg_flow_vjp(pffrg_ctx *ctx, int n_lambda, const double *lambdas, const double *d_checkpoints,
                            double *d_cot, double *d_dcoupling);

/* How the three channels of the vertex flow (Eq. 24) are launched; every
 * form computes dGamma = (s part + u part) + t part in that order, so the
 * results are bitwise the same:
 *   PFFRG_VERTEX_ONE_LAUNCH   one launch whose workgroups take the s, u and t
 *                             roles in turn, then the sum of the parts;
 *   PFFRG_VERTEX_SEPARATE     three launches in turn (s writes, u and t add);
 *   PFFRG_VERTEX_CONCURRENT   the t channel on the context's stream while s
 *                             and u run on a second stream of the context
 *                             (default priority), joined before the sum;
 *   PFFRG_VERTEX_AUTO         (the default) concurrent beyond 20 pairs, one
 *                             launch otherwise.
 * Profiling a single channel (PFFRG_K_VERTEX_S, _U, _T) uses the separate
 * form.  XYZ contexts run the concurrent form beyond 16 pairs when it is
 * chosen (explicitly, or by AUTO beyond 20) and the launches in turn
 * otherwise; TRI contexts always run them in turn.  An unknown mode gives
 * PFFRG_EINVAL. */
enum {
    PFFRG_VERTEX_AUTO = -1,
    PFFRG_VERTEX_ONE_LAUNCH = 0,
    PFFRG_VERTEX_SEPARATE = 1,
    PFFRG_VERTEX_CONCURRENT = 2
};
pffrg_status pffrg_set_vertex_mode(pffrg_ctx *ctx, int mode);

/* ----------------------------------------------------------- profiling - */

/* Kernel timing with HIP events on the context's stream for every launch of
 * the timed kernels (no effect on results).  The single-kernel ids get the
 * start and end of the launch itself (events handed to the launch, adding
 * nothing to the stream); PFFRG_K_VERTEX is timed by events recorded before
 * the first and after the last vertex launch (a few microseconds of stream
 * time each).  The vertex channels normally run as one launch
 * (PFFRG_K_VERTEX_STU) followed by the sum of the channel parts, or as
 * concurrent launches (pffrg_set_vertex_mode; PFFRG_K_VERTEX then spans the
 * fork to the join); while any of PFFRG_K_VERTEX_S, _U, _T is timed they run
 * as three launches in turn instead (the s launch writes, the u and t
 * launches add: the same sums, bitwise).
 * pffrg_set_profiling turns recording on
 * for all of them (1) or off (0); pffrg_set_profiling_mask records only the
 * kernels whose bit (1 << id) is set in `mask` (0: off; a bit at or above
 * PFFRG_K_COUNT: PFFRG_EINVAL).  Both synchronise the stream and clear the
 * totals.  pffrg_profile_read synchronises the stream and returns, for kernel
 * id `kernel`, the summed duration in milliseconds and the launch count since
 * profiling was switched on.  Up to 65536 launches per kernel are kept. */
enum {
    PFFRG_K_SIGMA = 0,      /* self-energy flow */
    PFFRG_K_TABLES = 1,     /* per-channel quadrature tables (with the packed vertex copy, same launch) */
    PFFRG_K_VERTEX = 2,     /* the whole vertex flow (all its launches) */
    PFFRG_K_VERTEX_S = 3,   /* s channel, own launch */
    PFFRG_K_VERTEX_U = 4,   /* u channel, own launch */
    PFFRG_K_VERTEX_T = 5,   /* t channel with the lattice sum, own launch */
    PFFRG_K_VERTEX_STU = 6, /* s, u and t channels in one launch (the default) */
    PFFRG_K_COUNT = 7
};
pffrg_status pffrg_set_profiling(pffrg_ctx *ctx, int on);
pffrg_status pffrg_set_profiling_mask(pffrg_ctx *ctx, unsigned mask);
pffrg_status pffrg_profile_read(pffrg_ctx *ctx, int kernel, double *total_ms, int *count);

/* ------------------------------------------------------------ batches -- */

/*
 * A batch advances n_points independent flows on one frequency mesh in
 * lockstep: the scans over couplings and lattice ranges with which phase
 * diagrams are mapped (Sec. 6.1, which also suggests reduced precision for
 * such scans).  Each point has its own lattice (at most 20 reduced pairs in
 * this kernel build) and flow state; mesh, precision and the RK4 cutoff
 * schedule are shared.  Per point the arithmetic is that of pffrg_rhs /
 * pffrg_step; the batch runs the self-energy flow, the quadrature tables and
 * the vertex flow of all points as single launches (the vertex one a
 * persistent kernel over a list of tiles of output triples) and can replay
 * one RK4 step as a hipGraph.
 *
 * Batch state: the points' states (single-flow layout) back to back; point
 * p starts at offsets[p] (in doubles) and offsets[n_points] is the total
 * size.  chi of a batch: the points' [2][Ns_p] arrays back to back.
 */
typedef struct pffrg_batch pffrg_batch;

/* lats[p] as for pffrg_create (host arrays, copied).  Errors as for
 * pffrg_create; a point with more than 20 pairs gives PFFRG_EUNSUPPORTED. */
pffrg_status pffrg_batch_create(int n_points, const pffrg_lattice *const *lats, const pffrg_mesh *mesh,
                                pffrg_precision prec, void *stream, pffrg_batch **out);
pffrg_status pffrg_batch_destroy(pffrg_batch *batch);

/* offsets[n_points + 1] (host) as described above. */
pffrg_status pffrg_batch_state_offsets(const pffrg_batch *batch, size_t *offsets);

/* Initial condition of every point (as pffrg_init_state). */
pffrg_status pffrg_batch_init_state(pffrg_batch *batch, double *d_state);

/* d_dstate = d state / d Lambda of every point at cutoff lambda > 0 (as
 * pffrg_rhs, Eq. 23 and Eq. 24).  d_state and d_dstate must not overlap. */
pffrg_status pffrg_batch_rhs(pffrg_batch *batch, double lambda, const double *d_state, double *d_dstate);

/* Classical RK4 (as pffrg_step with PFFRG_RK4) from lambdas[0] through
 * lambdas[n_lambda-1] (host array, 2 <= n_lambda <= 65536, all finite and
 * > 0) for every point, in place.  use_graph != 0 captures one step into a
 * hipGraph (once per state pointer and launch shape) and replays it; the
 * results are identical to use_graph == 0.  No observer runs; if
 * point_finite (host, [n_points]) is not NULL the call synchronises and
 * writes 1 for every point whose final state is finite, else 0 (points are
 * independent: a diverging point does not affect the others). */
pffrg_status pffrg_batch_flow(pffrg_batch *batch, int n_lambda, const double *lambdas, double *d_state,
                              int use_graph, int *point_finite);

/* chi per pair of every point (as pffrg_chi, Eq. 30), concatenated. */
pffrg_status pffrg_batch_chi(pffrg_batch *batch, double lambda, const double *d_state, double *d_chi);

/* chi(k) of point `point` (as pffrg_chi_k, Eq. 31) from its chi block. */
pffrg_status pffrg_batch_chi_k(pffrg_batch *batch, int point, const double *d_chi_point, int n_k,
                               const double *d_k, double *d_chi_k);

/* Launch shape of the persistent vertex kernel: `per` workgroups per XCD,
 * the tile order (0: each point's tiles on one XCD, chosen so the XCDs
 * carry equal estimated cost; 1: tiles dealt round-robin over the XCDs) and
 * split (0: one launch computes all three channels; 1: one launch for the s
 * and u channels, a second for the t channel, each with fewer registers).
 * pffrg_batch_tune times every candidate (per in 32, 64, 96, 128, 192, 256, 384, 512; both
 * orders; both splits) on three right-hand sides at (lambda, d_state),
 * keeps the fastest and caches it for the process under (n_freq, pair
 * counts, precision); a later batch with the same key starts with it.
 * Outputs may be NULL.  The shape never changes results. */
pffrg_status pffrg_batch_tune(pffrg_batch *batch, double lambda, const double *d_state, int *per, int *order,
                              int *split);
pffrg_status pffrg_batch_set_launch(pffrg_batch *batch, int per, int order, int split);

/* HIP-event timing of the vertex launch of direct (non-graph) batch right-
 * hand sides, as pffrg_set_profiling / pffrg_profile_read. */
pffrg_status pffrg_batch_set_profiling(pffrg_batch *batch, int on);
pffrg_status pffrg_batch_profile_read(pffrg_batch *batch, double *total_ms, int *count);

/* --------------------------------------------------------- diagnostics - */

/* Measured peaks of the device the stream (a hipStream_t or NULL) runs on,
 * for roofline fractions:
 * FP64 and FP32 vector FMA throughput (2 flops per FMA, every CU, 8
 * independent FMA chains per lane, FP32 without packed instructions as in
 * every kernel of the library) and the bandwidth of a 512 MiB device-to-
 * device copy (bytes read + written per second), and the rates at which 16
 * bytes per lane reach the registers, the width of one interpolation corner
 * of the vertex kernels (TB/s over every CU): 128-bit buffer loads from a
 * 16 KB L1-resident buffer, each wave instruction one contiguous 1 KB row
 * (l1_load_tbs) or two 512-byte rows (l1_load_2row_tbs, two pair vectors per
 * instruction), and 128-bit LDS reads (lds_read_tbs).  Allocates 1 GiB of
 * device memory for the duration of the call and frees it; synchronises the
 * stream.  Errors: PFFRG_EINVAL (NULL out), PFFRG_ENOMEM, PFFRG_EHIP. */
typedef struct pffrg_peaks {
    double fp64_fma_tflops;
    double fp32_fma_tflops;
    double hbm_copy_gbs;
    double l1_load_tbs;
    double l1_load_2row_tbs;
    double lds_read_tbs;
} pffrg_peaks;
pffrg_status pffrg_measure_peaks(void *stream, pffrg_peaks *out);

/* -------------------------------------------------------------- errors -- */

const char *pffrg_last_error(void);
const char *pffrg_status_string(pffrg_status s);

#ifdef __cplusplus
}
#endif

#endif /* PFFRG_H */
