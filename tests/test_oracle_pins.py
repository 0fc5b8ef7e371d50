"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the pin it implements; none compares the oracle with itself.
  lattice counts        the site counts the paper prints (tests/golden) and
                        closed forms of lattice balls
  initial condition     Sigma = 0, Gamma = J/4 (Eq. 14, Eq. 21)
  first right-hand side closed form of the flow at the initial condition,
                        derived by hand from Eq. 24 with the bare bubbles
  J = 0 fixed point     every right-hand side vanishes exactly
  two oracles           the C oracle (real SU(2)-reduced algebra) against the
                        literal spin-index evaluation with complex propagators
  SU(2) closure         off-diagonal basis functions stay zero, 11=22=33
  symmetry relations    the flow obeys Eq. 18 at arguments outside the octant
  Katanin quadrature    trapezoid on mesh nodes converges at second order to
                        an adaptive quadrature of the same integrand
  correlations          free-spin and first-order chi converge to their
                        continuum closed forms
  second order flow     the O(J^2) part of a flow equals the RK4 integral of
                        the closed-form first right-hand side
"""

import math
import os

import numpy as np
import pytest
from scipy import integrate

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _coupling_by_distance(lattice, params):
    shells = {"square": (("j1", 1.0), ("j2", math.sqrt(2)), ("j3", 2.0)),
              "honeycomb": (("j1", 1.0), ("j2", math.sqrt(3)), ("j3", 2.0))}[lattice]

    def J(r):
        d = float(np.linalg.norm(r))
        for name, dist in shells:
            if abs(d - dist) < 1e-9:
                return params.get(name, 0.0)
        return 0.0
    return J


def _brute_pair_sum(cell, J, r_i, r_k, reach=6):
    """sum over every lattice site j of J(r_j - r_i) J(r_k - r_j), brute force."""
    tot = 0.0
    for d0 in range(-reach, reach + 1):
        for d1 in range(-reach, reach + 1):
            for b in range(cell.n_basis):
                rj = cell.position((d0, d1, 0), b)
                tot += J(rj - r_i) * J(r_k - rj)
    return tot


# ------------------------------------------------------------ lattice ---

def test_lattice_counts_printed_in_paper(oracle_lib):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "lattice_counts.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        lat, L, ntot = r[0], int(r[1]), int(r[2])
        u = oracle_lib.sites.UnreducedLattice(W.model(lat, j1=1.0), L)
        assert all(int(n) == ntot for n in u.nsites), (lat, L, u.nsites)


@pytest.mark.parametrize("L", [1, 2, 3, 5, 7])
def test_lattice_balls_closed_form(oracle_lib, L):
    sq = oracle_lib.sites.UnreducedLattice(W.model("square", j1=1.0), L)
    assert sq.nsites[0] == 2 * L * L + 2 * L + 1
    # every listed site has Manhattan length <= L and the BFS distance equals it
    man = np.abs(sq.cell[0, :sq.nsites[0]]).sum(axis=1)
    assert np.array_equal(man, sq.dist[0, :sq.nsites[0]])
    if L <= 5:
        cu = oracle_lib.sites.UnreducedLattice(W.model("cubic", j1=1.0), L)
        assert cu.nsites[0] == (2 * L + 1) * (2 * L * L + 2 * L + 3) // 3


# ---------------------------------------------------- initial condition ---

def test_initial_condition(oracle_lib):
    m = W.model("honeycomb", j1=0.7, j2=0.2, j3=0.1)
    o = oracle_lib.Oracle(m, 3, W.log_mesh(0.01, 10.0, 5))
    x = o.initial_state()
    sig, gs, gd = o.split(x)
    J = _coupling_by_distance("honeycomb", m.params)
    assert np.all(sig == 0.0) and np.all(gd == 0.0)
    for b in range(o.lat.nb):
        for k in range(o.lat.nsites[b]):
            expect = J(o.lat.site_pos[b, k] - o.lat.basis_pos[b]) / 4.0
            assert np.all(gs[b, :, :, k] == expect)


# ------------------------------------------------ first RHS closed form ---

def _h(v, lam):
    return 1.0 / (v + lam) - (1.0 / (v - lam) if v > 2.0 * lam else 0.0)


@pytest.mark.parametrize("lattice,params,L", [
    ("square", dict(j1=1.0, j2=0.3), 3),
    ("honeycomb", dict(j1=1.0, j2=0.5, j3=0.25), 3),
])
@pytest.mark.parametrize("lam", [0.037, 0.41, 3.3, 60.0])
def test_first_rhs_closed_form(oracle_lib, lattice, params, L, lam):
    """At Sigma = 0, Gamma = J/4 the flow has no Katanin part (dSigma = 0) and
    every bubble is analytic.  With g = J/4 and
    h(v) = 1/(v+lam) - theta(v-2lam)/(v-lam):
      dGs_p = 2/(pi lam) [-g_p^2 (h(s)+h(u)) + (sum_j g_0j g_jp) h(t)]
      dGd_p = 3 g_p^2/(pi lam) [h(s) - h(u)]."""
    m = W.model(lattice, **params)
    mesh = W.log_mesh(0.005, 50.0, 7)
    o = oracle_lib.Oracle(m, L, mesh)
    d = o.rhs(lam, o.initial_state())
    sig, gs, gd = o.split(d)
    assert np.all(sig == 0.0)
    J = _coupling_by_distance(lattice, params)
    cell = W.unit_cell(lattice)
    err = 0.0
    for b in range(o.lat.nb):
        rb = o.lat.basis_pos[b]
        for k in range(o.lat.nsites[b]):
            rk = o.lat.site_pos[b, k]
            g = J(rk - rb) / 4.0
            sgg = _brute_pair_sum(cell, J, rb, rk) / 16.0
            for a in range(o.nf):
                for c in range(a + 1):
                    su = a * (a + 1) // 2 + c
                    for t in range(o.nf):
                        s_, u_, t_ = mesh[a], mesh[c], mesh[t]
                        es = 2.0 / (math.pi * lam) * (-g * g * (_h(s_, lam) + _h(u_, lam)) + sgg * _h(t_, lam))
                        ed = 3.0 * g * g / (math.pi * lam) * (_h(s_, lam) - _h(u_, lam))
                        err = max(err, abs(gs[b, su, t, k] - es), abs(gd[b, su, t, k] - ed))
    scale = max(np.abs(gs).max(), np.abs(gd).max())
    assert err <= 1e-14 * max(scale, 1.0), (err, scale)


# ------------------------------------------------------ J = 0 fixed point ---

def test_zero_coupling_is_a_fixed_point(oracle_lib):
    m = W.model("square", j1=0.0)
    o = oracle_lib.Oracle(m, 2, W.log_mesh(0.005, 50.0, 6))
    x = o.initial_state()
    x[: o.nf] = -np.linspace(0.1, 0.4, o.nf)      # any self-energy
    for lam in (0.01, 0.5, 20.0):
        assert np.all(o.rhs(lam, x) == 0.0)


# ----------------------------------------------------------- two oracles ---

def _random_oracle_state(o, seed):
    rng = np.random.default_rng(seed)
    x = o.initial_state()
    sig, gs, gd = o.split(x)
    sig[:] = -np.abs(rng.normal(0, 0.3, o.nf))
    gs[...] = rng.normal(0, 0.3, gs.shape)
    gd[...] = rng.normal(0, 0.3, gd.shape)
    for a in range(o.nf):
        gd[:, a * (a + 1) // 2 + a] = 0.0
    return x


@pytest.mark.parametrize("lattice,params", [("square", dict(j1=1.0)),
                                            ("honeycomb", dict(j1=1.0, j2=0.4))])
@pytest.mark.parametrize("lam", [0.03, 0.7, 2.2, "mesh"])
def test_c_oracle_matches_literal_spin_evaluation(oracle_lib, lattice, params, lam):
    from oracle.literal import LiteralFlow
    o = oracle_lib.Oracle(W.model(lattice, **params), 1, W.log_mesh(0.05, 5.0, 4))
    if lam == "mesh":          # cutoff on a mesh point: delta points hit theta ties
        lam = float(o.mesh[1])
    x = _random_oracle_state(o, 11)
    lf = LiteralFlow(o)
    ds_c = o.sigma_rhs(lam, x)
    ds_a = lf.sigma_rhs(lam, x)
    assert np.abs(ds_a.real).max() == 0.0                 # Sigma stays imaginary
    assert np.allclose(ds_c, ds_a.imag, rtol=0, atol=1e-14 * max(1, np.abs(ds_c).max()))
    full = o.rhs(lam, x)
    _, gs, gd = o.split(full)
    scale = max(np.abs(gs).max(), 1.0)
    closure = 0.0
    for b in range(o.lat.nb):
        for k in range(o.lat.nsites[b]):
            for a in range(o.nf):
                for c in range(a + 1):
                    for t in range(o.nf):
                        r = lf.vertex_rhs(lam, x, ds_c, b, k, a, t, c)
                        su = a * (a + 1) // 2 + c
                        assert abs(gs[b, su, t, k] - r[3, 3].real) <= 1e-13 * scale
                        assert abs(gd[b, su, t, k] - r[0, 0].real) <= 1e-13 * scale
                        off = r - np.diag(np.diag(r))
                        closure = max(closure, np.abs(r.imag).max(), np.abs(off).max(),
                                      abs(r[1, 1] - r[3, 3]), abs(r[2, 2] - r[3, 3]))
    # SU(2) closure: the flow of the off-diagonal / unequal components vanishes
    assert closure <= 1e-14 * scale
    zz, dd = o.chi(lam, x)
    for b in range(o.lat.nb):
        for k in range(o.lat.nsites[b]):
            assert abs(zz[b, k] - lf.chi(lam, x, b, k, 3).real) <= 1e-13
            assert abs(dd[b, k] - lf.chi(lam, x, b, k, 0).real) <= 1e-13


def test_flow_obeys_vertex_symmetry_relations(oracle_lib):
    """Eq. 18 holds for the computed flow at arguments outside the octant:
    s->-s and u->-u swap the sites (with mu<->nu), t->-t is free, and
    s<->u multiplies by -xi(nu).  Checked on the analytic (delta-function)
    part of every channel, which evaluates every vertex of Eq. 24 at exact
    points; the trapezoid of the Katanin part is not invariant under the
    substitutions that map the channels into each other, and the frequency
    window [-wmax, wmax] is not either, so that part obeys the relations only
    up to quadrature and truncation error."""
    from oracle.literal import LiteralFlow, XI
    o = oracle_lib.Oracle(W.model("honeycomb", j1=1.0, j2=0.4), 1, W.log_mesh(0.05, 5.0, 4))
    x = _random_oracle_state(o, 5)
    lam = 0.45
    ds = np.zeros(o.nf)
    lf = LiteralFlow(o)
    b, k = 0, 1
    dk = tuple(o.lat.cell[b, k]); bk = int(o.lat.bas[b, k])
    rev = tuple(-v for v in dk)
    s, t, u = 1.3, 0.6, 0.35
    base = lf.vertex_rhs_at(lam, x, ds, b, dk, bk, s, t, u)
    tol = 1e-13
    sw = lf.vertex_rhs_at(lam, x, ds, bk, rev, b, -s, t, u)
    assert np.abs(base - sw.T).max() < tol
    tm = lf.vertex_rhs_at(lam, x, ds, b, dk, bk, s, -t, u)
    assert np.abs(base - np.outer(XI, XI) * tm).max() < tol
    um = lf.vertex_rhs_at(lam, x, ds, bk, rev, b, s, t, -u)
    assert np.abs(base - np.outer(XI, XI) * um.T).max() < tol
    ex = lf.vertex_rhs_at(lam, x, ds, b, dk, bk, u, t, s)
    assert np.abs(base - (-XI)[None, :] * ex).max() < tol


# --------------------------------------------------- Katanin quadrature ---

def _odd_interp(mesh, vals, w):
    sgn = -1.0 if w < 0 else 1.0
    return sgn * np.interp(abs(w), mesh, vals)   # constant outside the mesh


def test_katanin_trapezoid_converges_second_order(oracle_lib):
    """Isolate the Katanin term (difference of two right-hand sides that
    differ only in dSigma), for a frequency-independent spin vertex, and
    compare it with an adaptive quadrature of the same interpolated
    integrand over the same domain.  The error must fall ~4x per mesh
    doubling (trapezoid rule, Sec. 4.2)."""
    m = W.model("square", j1=1.0)
    lam = 0.3
    phi = lambda w: -0.3 * w / (1.0 + w * w)
    psi = lambda w: 0.5 * w / (1.0 + w * w) ** 2
    cvals = {0: 0.21, 1: 0.25}                      # onsite, nearest neighbour (Gs)
    errs = []
    for n in (24, 48, 96):
        mesh = W.log_mesh(0.01, 20.0, n)
        o = oracle_lib.Oracle(m, 1, mesh)
        x = o.initial_state()
        sig, gs, gd = o.split(x)
        sig[:] = phi(mesh)
        dist = o.lat.dist[0]
        for k in range(o.lat.nsites[0]):
            gs[0, :, :, k] = cvals[int(dist[k])]
        dsig = psi(mesh)
        a, t, c = n - 1 - n // 3, n // 2, n // 4
        k = 1
        kat = (o.vertex_rhs_element(lam, x, dsig, 0, k, a, t, c)
               - o.vertex_rhs_element(lam, x, np.zeros(n), 0, k, a, t, c))
        s_, t_, u_ = mesh[a], mesh[t], mesh[c]
        cp, c0 = cvals[1], cvals[0]
        # square lattice, range 1: sum_j G_0j G_jk over j in range of both ends
        sgg = 2 * c0 * cp   # j = 0 and j = k (only those are within one bond of both)
        F = {"s": (-2 * cp * cp, 3 * cp * cp), "t": (-2 * sgg - 2 * cp * c0, 0.0),
             "u": (2 * cp * cp, 3 * cp * cp)}
        g = lambda w: 1.0 / (w - _odd_interp(mesh, sig, w))
        ps = lambda w: _odd_interp(mesh, dsig, w)
        wmax = mesh[-1]
        expect = np.zeros(2)
        for ch, part, cen in (("s", lambda w: s_ - w, s_), ("t", lambda w: w - t_, t_),
                              ("u", lambda w: u_ + w, -u_)):
            f = lambda w, p=part: g(w) * g(p(w)) ** 2 * ps(p(w)) + g(p(w)) * g(w) ** 2 * ps(w)
            cuts = sorted({-lam, lam, cen - lam, cen + lam})
            brk = sorted(set(list(mesh) + list(-mesh) + [cen - v for v in mesh] + [cen + v for v in mesh]))
            edges = [-wmax] + [v for v in cuts if -wmax < v < wmax] + [wmax]
            for lo, hi in zip(edges[:-1], edges[1:]):
                mid = 0.5 * (lo + hi)
                if abs(mid) < lam or abs(part(mid)) < lam or hi <= lo:
                    continue
                pts = [v for v in brk if lo < v < hi]
                val, _ = integrate.quad(f, lo, hi, points=pts[:400] if pts else None,
                                        limit=2000, epsabs=1e-13, epsrel=1e-12)
                expect += np.array(F[ch]) * val / (2 * math.pi)
        errs.append(np.abs(kat - expect).max() / np.abs(expect).max())
    assert errs[2] < 1e-2
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 2.5, errs


# ----------------------------------------------------------- correlations ---

def test_free_spin_and_first_order_chi_converge(oracle_lib):
    """J=0: chi_ii -> (1/2pi)(1/lam - 1/wmax) (a free spin, truncated at wmax).
    Initial condition: chi_ij -> -(J_ij/(4 pi^2)) (1/lam - 1/wmax)^2."""
    lam, wmax, J = 0.2, 30.0, 0.8
    free_exact = (1.0 / lam - 1.0 / wmax) / (2 * math.pi)
    first_exact = -J / (4 * math.pi ** 2) * (1.0 / lam - 1.0 / wmax) ** 2
    e1, e2 = [], []
    for n in (32, 64, 128):
        mesh = W.log_mesh(0.01, wmax, n)
        o0 = oracle_lib.Oracle(W.model("square", j1=0.0), 1, mesh)
        zz, dd = o0.chi(lam, o0.initial_state())
        assert np.all(zz[0, 1:] == 0.0) and zz[0, 0] == dd[0, 0]
        e1.append(abs(zz[0, 0] - free_exact) / free_exact)
        oj = oracle_lib.Oracle(W.model("square", j1=J), 1, mesh)
        zz, dd = oj.chi(lam, oj.initial_state())
        e2.append(abs(zz[0, 1] - first_exact) / abs(first_exact))
    for e in (e1, e2):
        assert e[2] < 5e-3 and e[0] / e[1] > 3.0 and e[1] / e[2] > 3.0, e


# ------------------------------------------------------ second-order flow ---

def test_flow_second_order_perturbation_theory(oracle_lib):
    """Scale J -> eps J.  To O(eps^2) the vertex obeys the closed-form first
    right-hand side with g frozen at eps J/4 (Sigma and the Katanin term enter
    at higher order), so (Gamma(lam_f) - eps J/4)/eps^2 from an RK4 flow must
    equal the RK4 integral of that closed form up to O(eps)."""
    mesh = W.log_mesh(0.01, 20.0, 5)
    sched = W.geometric_schedule(20.0, 0.5, 6)
    L = 2
    base = {"j1": 1.0, "j2": 0.4}
    J = _coupling_by_distance("square", base)
    cell = W.unit_cell("square")
    res = []
    for eps in (2e-3, 1e-3):
        o = oracle_lib.Oracle(W.model("square", **{k: eps * v for k, v in base.items()}), L, mesh)
        x = o.flow(sched)
        _, gs, gd = o.split(x - o.initial_state())
        res.append((gs / eps ** 2, gd / eps ** 2))
    o = oracle_lib.Oracle(W.model("square", **base), L, mesh)

    def closed(lam):
        out_s = np.zeros_like(res[0][0]); out_d = np.zeros_like(res[0][1])
        for k in range(o.lat.nsites[0]):
            rk = o.lat.site_pos[0, k]
            g = J(rk) / 4.0
            sgg = _brute_pair_sum(cell, J, np.zeros(3), rk) / 16.0
            for a in range(o.nf):
                for c in range(a + 1):
                    su = a * (a + 1) // 2 + c
                    for t in range(o.nf):
                        s_, u_, t_ = mesh[a], mesh[c], mesh[t]
                        out_s[0, su, t, k] = 2 / (math.pi * lam) * (-g * g * (_h(s_, lam) + _h(u_, lam)) + sgg * _h(t_, lam))
                        out_d[0, su, t, k] = 3 * g * g / (math.pi * lam) * (_h(s_, lam) - _h(u_, lam))
        return out_s, out_d

    ys = np.zeros_like(res[0][0]); yd = np.zeros_like(res[0][1])
    for i in range(len(sched) - 1):
        l0, l1 = sched[i], sched[i + 1]
        hh = l1 - l0
        k1, k2, k4 = closed(l0), closed(l0 + 0.5 * hh), closed(l1)
        ys = ys + hh / 6 * (k1[0] + 4 * k2[0] + k4[0])
        yd = yd + hh / 6 * (k1[1] + 4 * k2[1] + k4[1])
    d1 = max(np.abs(res[0][0] - ys).max(), np.abs(res[0][1] - yd).max())
    d2 = max(np.abs(res[1][0] - ys).max(), np.abs(res[1][1] - yd).max())
    scale = np.abs(ys).max()
    assert d2 < 1e-2 * scale
    assert 1.6 < d1 / d2 < 2.4, (d1, d2)      # the remainder is O(eps)
