"""Pins of the oracle's structure factor and integrators.

Each test checks the oracle against what the paper and the mathematics fix,
never against a second transcription of the same code:
  structure factor      Eq. 31 evaluated by brute force over every site pair
                        of a periodic cluster (no site lists of the oracle),
                        and the flat J = 0 result
  Dormand-Prince step   fifth-order global convergence and a fifth-order
                        embedded error estimate on an ODE with a closed-form
                        solution (any wrong tableau entry or a missing
                        dx/dl = Lambda dx/dLambda factor breaks one of them)
  adaptive controller   tolerance met on that ODE, steps ending on each side
                        of every breakpoint
  adaptive / Euler flow the O(J^2) part of a flow equals the exact integral
                        (adaptive) or the Euler sum (Euler, Eq. 42) of the
                        closed-form first right-hand side, up to O(J)
"""

import math
from collections import deque

import numpy as np
import pytest
from scipy import integrate

import workloads as W


# --------------------------------------------------- structure factor ---

def _phi(b1, b2, d):
    """A correlation chi_ij that depends on the two sublattices and on
    d = r_j - r_i, symmetric under exchanging i and j (as chi_ij = chi_ji)."""
    def psi(x1, x2, e):
        return (math.cos(0.7 * e[0] + 1.3 * e[1] + 0.4 * e[2] + 0.9 * x1 - 0.2 * x2 + 0.3)
                * math.exp(-0.15 * float(e @ e)) + 0.05 * x1)
    return psi(b1, b2, d) + psi(b2, b1, -d)


def _cluster_structure_factor(cell, L, n, dims, kpts):
    """chi(k) of Eq. 31 on an n^dims-cell periodic cluster:
    (1/N_L) sum_{i,j} exp(i k (r_i - r_j)) sum_mu chi^{mu mu}_ij with
    sum_mu chi^{mu mu} = 3 chi^{zz} (SU(2)), chi^{zz}_ij = _phi for every j
    within L bonds of i (found by breadth-first search on the cluster's own
    bond graph) and 0 beyond.  k must lie on the cluster's reciprocal grid."""
    nb = cell.n_basis
    nbrs = [[] for _ in range(nb)]
    for (f, t, d0, d1, d2) in cell.bonds:
        nbrs[f].append((np.array([d0, d1, d2]), t))
        nbrs[t].append((-np.array([d0, d1, d2]), f))

    def wrap(c):
        c = np.array(c)
        c[:dims] %= n
        return tuple(int(v) for v in c)

    cells = [tuple(int(v) for v in c) for c in np.ndindex(*([n] * dims + [1] * (3 - dims)))]
    sites = [(c, b) for c in cells for b in range(nb)]
    pos = {s: np.array(s[0], dtype=float) @ cell.primitives + cell.basis[s[1]] for s in sites}
    tot = np.zeros(len(kpts), dtype=complex)
    for (ci, bi) in sites:
        # unwrapped offsets along the search; the cluster is large enough when
        # no site of the ball is reached through two different offsets
        start = (np.zeros(3, dtype=int), bi)
        seen = {(wrap(np.array(ci)), bi): (0, tuple(start[0]))}
        q = deque([start])
        while q:
            off, b = q.popleft()
            dist = seen[(wrap(np.array(ci) + off), b)][0]
            if dist == L:
                continue
            for (d, b2) in nbrs[b]:
                o2 = off + d
                key = (wrap(np.array(ci) + o2), b2)
                if key in seen:
                    assert seen[key][1] == tuple(o2), "cluster too small"
                    continue
                seen[key] = (dist + 1, tuple(o2))
                q.append((o2, b2))
        ri = pos[(ci, bi)]
        for (cj, bj), (_, off) in seen.items():
            off = np.array(off)
            d = off @ cell.primitives + cell.basis[bj] - cell.basis[bi]
            rj = pos[(cj, bj)]
            tot += np.exp(1j * (kpts @ (ri - rj))) * 3.0 * _phi(bi, bj, d)
    return tot / len(sites)


@pytest.mark.parametrize("lattice,L,n,dims", [
    ("square", 3, 8, 2),
    ("honeycomb", 4, 10, 2),
    ("pyrochlore", 2, 6, 3),
])
def test_structure_factor_brute_force_cluster(oracle_lib, lattice, L, n, dims):
    """Eq. 31 with the normalisation by the number of sites summed over: the
    oracle's per-unit-cell form (1/N_b) sum_b sum_{j in range of b} must give
    the cluster sum exactly at every k of the cluster's reciprocal grid."""
    cell = W.unit_cell(lattice)
    o = oracle_lib.Oracle(W.model(lattice, j1=1.0), L, W.log_mesh(0.1, 10.0, 2))
    lat = o.lat
    zz = np.zeros((lat.nb, lat.ns))
    for b in range(lat.nb):
        for j in range(lat.nsites[b]):
            zz[b, j] = _phi(b, int(lat.bas[b, j]), lat.site_pos[b, j] - lat.basis_pos[b])
    g = np.linalg.inv(cell.primitives).T            # rows: reciprocal vectors / 2 pi
    rng = np.random.default_rng(2109)
    ms = [np.zeros(3, dtype=int)] + [np.concatenate([rng.integers(0, n, dims), np.zeros(3 - dims, dtype=int)])
                                     for _ in range(6)]
    kpts = np.array([2.0 * math.pi * (m / n) @ g for m in ms])
    brute = _cluster_structure_factor(cell, L, n, dims, kpts)
    assert np.abs(brute.imag).max() < 1e-12
    got = o.chi_k(zz, kpts)
    scale = np.abs(brute.real).max()
    assert np.abs(got - brute.real).max() <= 1e-12 * scale, (got, brute.real)


def test_structure_factor_is_flat_at_zero_coupling(oracle_lib):
    """J = 0: only the on-site correlation survives, so chi(k) = 3 chi_ii for
    every k, on every sublattice (honeycomb: two basis sites)."""
    o = oracle_lib.Oracle(W.model("honeycomb", j1=0.0), 3, W.log_mesh(0.01, 30.0, 16))
    zz, _ = o.chi(0.3, o.initial_state())
    kpts = np.random.default_rng(5).uniform(-7.0, 7.0, size=(9, 3))
    got = o.chi_k(zz, kpts)
    assert zz[0, 0] == zz[1, 0] > 0.0
    assert np.abs(got - 3.0 * zz[0, 0]).max() <= 1e-14 * zz[0, 0]


# ------------------------------------------------------- Dormand-Prince ---

def _ode(lam, x):
    """dx/dLambda of a two-component ODE with a closed-form solution."""
    return np.array([x[0] ** 2 / lam, math.cos(lam)])


def _ode_exact(lam, lam0, x0):
    l, l0 = math.log(lam), math.log(lam0)
    return np.array([1.0 / (1.0 / x0[0] - (l - l0)), x0[1] + math.sin(lam) - math.sin(lam0)])


X0 = np.array([0.3, 0.1])


def test_dopri_step_fifth_order(oracle_lib):
    """n equal steps in ln Lambda: the global error falls by 2^5 per halving
    of the step."""
    lam0, lam1 = 4.0, 0.25
    exact = _ode_exact(lam1, lam0, X0)
    errs = []
    for n in (32, 64, 128):
        dl = (math.log(lam1) - math.log(lam0)) / n
        x, l = X0.copy(), math.log(lam0)
        for _ in range(n):
            x, _, _ = oracle_lib.dopri_step(_ode, l, dl, x, _ode(math.exp(l), x))
            l += dl
        errs.append(np.abs(x - exact).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    # 2^5 = 32 (reached from above); fourth order would give 16, sixth 64
    assert 28.0 < r1 < 42.0 and 28.0 < r2 < 42.0, errs


def test_dopri_embedded_estimate_fifth_order(oracle_lib):
    """One step: the embedded difference e = y5 - y4 is the local error of the
    fourth-order point, O(h^5), while y5 is accurate to O(h^6)."""
    lam0 = 2.0
    es, e5 = [], []
    for dl in (-0.1, -0.05, -0.025):
        y, e, k = oracle_lib.dopri_step(_ode, math.log(lam0), dl, X0, _ode(lam0, X0))
        exact = _ode_exact(lam0 * math.exp(dl), lam0, X0)
        es.append(np.abs(e).max())
        e5.append(np.abs(y - exact).max())
        # the last stage is the derivative at the new point (first same as last)
        assert np.array_equal(k[6], _ode(math.exp(math.log(lam0) + dl), y))
    assert 24.0 < es[0] / es[1] < 42.0 and 24.0 < es[1] / es[2] < 42.0, es
    assert e5[2] < 0.1 * es[2], (e5, es)
    assert e5[1] / e5[2] > 40.0, e5


def test_dopri_controller_meets_tolerance_and_lands_on_breakpoints(oracle_lib):
    brk = [2.5, 1.0, 0.4]
    seen = []
    x, lams = oracle_lib.dopri_integrate(_ode, X0, 4.0, 0.25, 1e-10, 1e-12, 0.05, 1e-9,
                                         breakpoints=brk, observer=lambda lam, y: seen.append(lam))
    exact = _ode_exact(0.25, 4.0, X0)
    assert np.abs(x - exact).max() <= 1e-8 * np.abs(exact).max()
    assert seen == lams and abs(lams[-1] - 0.25) <= 1e-15
    assert all(a > b for a, b in zip(lams, lams[1:]))
    # a step ends 1e-12 (in ln Lambda) above each breakpoint and the flow
    # continues from 1e-12 below it: an accepted cutoff sits there, and no
    # accepted step crosses a breakpoint anywhere else
    ll = np.log(np.array([4.0] + lams))
    for b in brk:
        lb = math.log(b)
        assert np.abs(ll - (lb - 1e-12)).min() < 1e-14
        for l0, l1 in zip(ll, ll[1:]):
            if l1 < lb < l0:
                assert abs(l1 - (lb - 1e-12)) < 1e-14 and l0 - lb > 1e-13
    # a looser tolerance takes fewer steps and is still met
    x2, lams2 = oracle_lib.dopri_integrate(_ode, X0, 4.0, 0.25, 1e-6, 1e-9, 0.05, 1e-9, breakpoints=brk)
    assert len(lams2) < len(lams)
    assert np.abs(x2 - exact).max() <= 1e-4 * np.abs(exact).max()


# ---------------------------------------- O(J^2) through the integrators ---

def _h(v, lam):
    return 1.0 / (v + lam) - (1.0 / (v - lam) if v > 2.0 * lam else 0.0)


def _coupling(params):
    shells = (("j1", 1.0), ("j2", math.sqrt(2)), ("j3", 2.0))

    def J(r):
        d = float(np.linalg.norm(r))
        for name, dist in shells:
            if abs(d - dist) < 1e-9:
                return params.get(name, 0.0)
        return 0.0
    return J


def _pair_sum(J, r_k, reach=6):
    """sum over all square-lattice sites j of J(r_j) J(r_k - r_j)."""
    tot = 0.0
    for d0 in range(-reach, reach + 1):
        for d1 in range(-reach, reach + 1):
            rj = np.array([d0, d1, 0.0])
            tot += J(rj) * J(r_k - rj)
    return tot


def _second_order_flows(oracle_lib, run, mesh, base, L=2):
    """(Gamma(end) - Gamma0)/eps^2 of the flows run(o) for eps = 2e-3, 1e-3."""
    out = []
    for eps in (2e-3, 1e-3):
        o = oracle_lib.Oracle(W.model("square", **{k: eps * v for k, v in base.items()}), L, mesh)
        x = run(o)
        _, gs, gd = o.split(x - o.initial_state())
        out.append((gs / eps ** 2, gd / eps ** 2))
    return out, oracle_lib.Oracle(W.model("square", **base), L, mesh)


def _closed_form(o, mesh, J, hfun):
    """Closed-form first right-hand side with h(v) replaced by hfun(v):
    dGs = (2/pi) [-g^2 (H(s) + H(u)) + (sum_j g g) H(t)], dGd = (3 g^2/pi) [H(s) - H(u)]."""
    gs = np.zeros((1, o.n_su, o.nf, o.lat.ns)); gd = np.zeros_like(gs)
    H = {i: hfun(float(mesh[i])) for i in range(o.nf)}
    for k in range(o.lat.nsites[0]):
        rk = o.lat.site_pos[0, k]
        g = J(rk) / 4.0
        sgg = _pair_sum(J, rk) / 16.0
        for a in range(o.nf):
            for c in range(a + 1):
                su = a * (a + 1) // 2 + c
                for t in range(o.nf):
                    gs[0, su, t, k] = 2 / math.pi * (-g * g * (H[a] + H[c]) + sgg * H[t])
                    gd[0, su, t, k] = 3 * g * g / math.pi * (H[a] - H[c])
    return gs, gd


def _check_remainder_is_first_order(res, ys, yd):
    d1 = max(np.abs(res[0][0] - ys).max(), np.abs(res[0][1] - yd).max())
    d2 = max(np.abs(res[1][0] - ys).max(), np.abs(res[1][1] - yd).max())
    scale = np.abs(ys).max()
    assert d2 < 1e-2 * scale, (d2, scale)
    assert 1.6 < d1 / d2 < 2.4, (d1, d2)      # the remainder is O(eps)


def test_adaptive_flow_second_order_perturbation_theory(oracle_lib):
    """Scale J -> eps J.  To O(eps^2) the vertex flows with the closed-form
    first right-hand side (g frozen at eps J/4), whose integral from Lambda_i
    to Lambda_f is H(v) = int h(v, Lambda)/Lambda dLambda per transfer
    frequency, computed here by adaptive quadrature split at the jump
    Lambda = v/2.  A tight adaptive Dormand-Prince flow must reproduce it up
    to O(eps)."""
    mesh = W.log_mesh(0.01, 20.0, 5)
    base = {"j1": 1.0, "j2": 0.4}
    lam_i, lam_f = 20.0, 0.5
    res, o = _second_order_flows(
        oracle_lib, lambda o: o.dopri_flow(lam_i, lam_f, 1e-9, 1e-16, 0.05, 1e-12)[0], mesh, base)

    def H(v):
        pts = [0.5 * v] if lam_f < 0.5 * v < lam_i else None
        val, _ = integrate.quad(lambda lam: _h(v, lam) / lam, lam_f, lam_i, points=pts,
                                epsabs=1e-15, epsrel=1e-13, limit=400)
        return -val
    ys, yd = _closed_form(o, mesh, _coupling(base), H)
    _check_remainder_is_first_order(res, ys, yd)


def test_euler_flow_second_order_perturbation_theory(oracle_lib):
    """Euler steps (Eq. 42) take the derivative at the start of each step, so
    the O(eps^2) part of the flow is the left Riemann sum of the closed-form
    first right-hand side over the schedule, up to O(eps)."""
    mesh = W.log_mesh(0.01, 20.0, 5)
    base = {"j1": 1.0, "j2": 0.4}
    sched = W.geometric_schedule(20.0, 0.5, 6)
    res, o = _second_order_flows(oracle_lib, lambda o: o.flow(sched, scheme="euler"), mesh, base)
    J = _coupling(base)
    ys = np.zeros_like(res[0][0]); yd = np.zeros_like(res[0][1])
    for i in range(len(sched) - 1):
        l0, l1 = float(sched[i]), float(sched[i + 1])
        ks, kd = _closed_form(o, mesh, J, lambda v: _h(v, l0) / l0)
        ys += (l1 - l0) * ks
        yd += (l1 - l0) * kd
    _check_remainder_is_first_order(res, ys, yd)
