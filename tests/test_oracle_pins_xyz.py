"""Pins of the oracle's XYZ form (couplings Jx S^x S^x + Jy S^y S^y +
Jz S^z S^z, Sec. 2; only the diagonal vertex components are non-zero, Sec. 3).

  first right-hand side   closed form at Sigma = 0, Gamma^mu = J^mu/4,
                          derived by hand from Eq. 24 with the bare bubbles
                          (the XYZ analogue of the SU(2) pin)
  SU(2) limit             Jx = Jy = Jz: the four-strain flow and correlations
                          equal the two-strain (SU(2)) ones, strain by strain
  literal evaluation      the C oracle against the explicit spin-index
                          equations with 2x2 spin tensors (oracle/literal.py):
                          right-hand side and chi per component, and XYZ
                          closure (off-diagonal components do not flow)
  J = 0                   every right-hand side vanishes exactly
"""

import math

import numpy as np
import pytest

import workloads as W


def _h(v, lam):
    return 1.0 / (v + lam) - (1.0 / (v - lam) if v > 2.0 * lam else 0.0)


SHELLS = {"square": (("j1", 1.0), ("j2", math.sqrt(2)), ("j3", 2.0)),
          "honeycomb": (("j1", 1.0), ("j2", math.sqrt(3)), ("j3", 2.0))}


def _coupling_by_distance(lattice, params):
    def J(r):
        d = float(np.linalg.norm(r))
        for name, dist in SHELLS[lattice]:
            if abs(d - dist) < 1e-9:
                return np.asarray(params.get(name, (0.0, 0.0, 0.0)), dtype=float)
        return np.zeros(3)
    return J


def _brute_pair_sum(cell, J, r_i, r_k, reach=6):
    """sum over every lattice site j of J^mu(r_j - r_i) J^mu(r_k - r_j), per mu."""
    tot = np.zeros(3)
    for d0 in range(-reach, reach + 1):
        for d1 in range(-reach, reach + 1):
            for b in range(cell.n_basis):
                rj = cell.position((d0, d1, 0), b)
                tot += J(rj - r_i) * J(r_k - rj)
    return tot


@pytest.mark.parametrize("lattice,params,L", [
    ("square", dict(j1=(1.0, 0.6, 0.3), j2=(0.2, -0.5, 0.4)), 3),
    ("honeycomb", dict(j1=(0.8, 1.0, -0.3), j2=(0.1, 0.25, 0.2), j3=(0.3, 0.0, 0.15)), 3),
])
@pytest.mark.parametrize("lam", [0.037, 0.41, 3.3])
def test_xyz_first_rhs_closed_form(oracle_lib, lattice, params, L, lam):
    """At Sigma = 0, Gamma^mu = g^mu = J^mu/4 (Gamma^d = 0) the flow has no
    Katanin part and every bubble is analytic: B_s(v) = h(v)/(pi lam),
    B_t = B_u = -h/(pi lam).  With the XYZ channel algebra of Eq. 24 ((a,b,c)
    cyclic in (x,y,z)):
      dGa_p = (1/(pi lam)) [-2 g^b g^c (h(s) + h(u)) + 2 h(t) sum_j g^a_0j g^a_jp]
      dGd_p = ((g^x^2 + g^y^2 + g^z^2)/(pi lam)) [h(s) - h(u)]."""
    m = W.model_xyz(lattice, **params)
    mesh = W.log_mesh(0.005, 50.0, 6)
    o = oracle_lib.Oracle(m, L, mesh)
    assert o.nc == 4
    d = o.rhs(lam, o.initial_state())
    sig, gx, gy, gz, gd = o.split(d)
    assert np.all(sig == 0.0)
    J = _coupling_by_distance(lattice, params)
    cell = W.unit_cell(lattice)
    got = (gx, gy, gz)
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
                        hs, hu, ht = _h(mesh[a], lam), _h(mesh[c], lam), _h(mesh[t], lam)
                        for mu in range(3):
                            nb_, nc_ = (mu + 1) % 3, (mu + 2) % 3
                            e = (-2.0 * g[nb_] * g[nc_] * (hs + hu) + 2.0 * ht * sgg[mu]) / (math.pi * lam)
                            err = max(err, abs(got[mu][b, su, t, k] - e))
                        ed = float(g @ g) / (math.pi * lam) * (hs - hu)
                        err = max(err, abs(gd[b, su, t, k] - ed))
    scale = max(np.abs(d).max(), 1.0)
    assert err <= 1e-14 * scale, (err, scale)


def _embed(o2, o4, x2):
    """The XYZ state with Gx = Gy = Gz = Gs and the same Gd and sigma."""
    x4 = np.zeros(o4.size)
    sig2, gs, gd = o2.split(x2)
    sig4, gx, gy, gz, gd4 = o4.split(x4)
    sig4[:] = sig2
    gx[...] = gs; gy[...] = gs; gz[...] = gs
    gd4[...] = gd
    return x4


@pytest.mark.parametrize("lattice,L", [("square", 2), ("honeycomb", 2)])
def test_xyz_reduces_to_su2(oracle_lib, lattice, L):
    """Jx = Jy = Jz = J and Gx = Gy = Gz: the XYZ flow keeps the three spin
    strains equal to the SU(2) spin strain and the density strain equal to
    the SU(2) one (up to rounding: the sums run in another order); so do the
    correlations."""
    j = dict(j1=1.0, j2=0.35)
    mesh = W.log_mesh(0.01, 20.0, 5)
    o2 = oracle_lib.Oracle(W.model(lattice, **j), L, mesh)
    o4 = oracle_lib.Oracle(W.model_xyz(lattice, **{k: (v, v, v) for k, v in j.items()}), L, mesh)
    rng = np.random.default_rng(3)
    x2 = o2.initial_state()
    sig, gs, gd = o2.split(x2)
    sig[:] = -np.abs(rng.normal(0, 0.3, o2.nf))
    gs += rng.normal(0, 0.3, gs.shape)
    gd[...] = rng.normal(0, 0.3, gd.shape)
    for a in range(o2.nf):
        gd[:, a * (a + 1) // 2 + a] = 0.0
    x4 = _embed(o2, o4, x2)
    assert np.array_equal(o4.initial_state(), _embed(o2, o4, o2.initial_state()))
    for lam in (0.02, 0.6, 4.0):
        d2 = o2.rhs(lam, x2)
        d4 = o4.rhs(lam, x4)
        ref = _embed(o2, o4, d2)
        scale = np.abs(d2).max()
        assert np.abs(d4 - ref).max() <= 1e-13 * scale, lam
        c2 = o2.chi_comps(lam, x2)
        c4 = o4.chi_comps(lam, x4)
        cs = np.abs(c2).max()
        for m4, m2 in ((0, 0), (1, 0), (2, 0), (3, 1)):
            assert np.abs(c4[m4] - c2[m2]).max() <= 1e-13 * cs, (lam, m4)


def _random_xyz_state(o, seed):
    rng = np.random.default_rng(seed)
    x = o.initial_state()
    sig, gx, gy, gz, gd = o.split(x)
    sig[:] = -np.abs(rng.normal(0, 0.3, o.nf))
    for g in (gx, gy, gz, gd):
        g[...] = rng.normal(0, 0.3, g.shape)
    for a in range(o.nf):
        gd[:, a * (a + 1) // 2 + a] = 0.0     # the s <-> u relation forces Gd(s, t, s) = 0
    return x


@pytest.mark.parametrize("lattice,params", [("square", dict(j1=(1.0, 0.5, 0.2))),
                                            ("honeycomb", dict(j1=(0.7, 1.0, 0.4), j2=(0.3, 0.2, 0.1)))])
@pytest.mark.parametrize("lam", [0.03, 0.7, "mesh"])
def test_xyz_c_oracle_matches_literal_spin_evaluation(oracle_lib, lattice, params, lam):
    from oracle.literal import LiteralFlow
    o = oracle_lib.Oracle(W.model_xyz(lattice, **params), 1, W.log_mesh(0.05, 5.0, 4))
    if lam == "mesh":
        lam = float(o.mesh[1])
    x = _random_xyz_state(o, 17)
    lf = LiteralFlow(o)
    ds_c = o.sigma_rhs(lam, x)
    ds_a = lf.sigma_rhs(lam, x)
    assert np.abs(ds_a.real).max() == 0.0
    assert np.allclose(ds_c, ds_a.imag, rtol=0, atol=1e-14 * max(1, np.abs(ds_c).max()))
    full = o.rhs(lam, x)
    _, gx, gy, gz, gd = o.split(full)
    comps = ((gd, 0), (gx, 1), (gy, 2), (gz, 3))        # (C strain, Pauli index)
    scale = max(np.abs(full).max(), 1.0)
    closure = 0.0
    for b in range(o.lat.nb):
        for k in range(o.lat.nsites[b]):
            for a in range(o.nf):
                for c in range(a + 1):
                    for t in range(o.nf):
                        r = lf.vertex_rhs(lam, x, ds_c, b, k, a, t, c)
                        su = a * (a + 1) // 2 + c
                        for g, mu in comps:
                            assert abs(g[b, su, t, k] - r[mu, mu].real) <= 1e-13 * scale
                        off = r - np.diag(np.diag(r))
                        closure = max(closure, np.abs(r.imag).max(), np.abs(off).max())
    # XYZ closure: off-diagonal components do not flow
    assert closure <= 1e-14 * scale
    chi = o.chi_comps(lam, x)
    for b in range(o.lat.nb):
        for k in range(o.lat.nsites[b]):
            for m, mu in ((0, 1), (1, 2), (2, 3), (3, 0)):
                assert abs(chi[m, b, k] - lf.chi(lam, x, b, k, mu).real) <= 1e-13


def test_xyz_zero_coupling_is_a_fixed_point(oracle_lib):
    o = oracle_lib.Oracle(W.model_xyz("square", j1=(0.0, 0.0, 0.0)), 2, W.log_mesh(0.005, 50.0, 5))
    x = o.initial_state()
    x[: o.nf] = -np.linspace(0.1, 0.4, o.nf)
    for lam in (0.01, 0.5, 20.0):
        assert np.all(o.rhs(lam, x) == 0.0)


def _coupling_by_bonds(model):
    """J^mu(r_i, r_j) of a model whose couplings depend on the bond: every
    listed interaction (param, b0, b1, d) joins the site of sublattice b0 in
    any cell R with the site of sublattice b1 in cell R + d (and back)."""
    cell = model.cell
    P = np.asarray(cell.primitives, dtype=float)
    B = np.asarray(cell.basis, dtype=float)
    inv = np.linalg.inv(P)

    def sub(r):
        for b in range(len(B)):
            f = (r - B[b]) @ inv
            if np.abs(f - np.rint(f)).max() < 1e-9:
                return b
        raise ValueError("not a lattice site")

    def J(ri, rj):
        bi, bj = sub(ri), sub(rj)
        tot = np.zeros(3)
        for (name, b0, b1, d0, d1, d2) in model.interactions:
            v = np.asarray(model.params[name], dtype=float)
            dr = np.array([d0, d1, d2], dtype=float) @ P + B[b1] - B[b0]
            if bi == b0 and bj == b1 and np.abs(rj - ri - dr).max() < 1e-9:
                tot += v
            if bi == b1 and bj == b0 and np.abs(ri - rj - dr).max() < 1e-9:
                tot += v
        return tot
    return J


@pytest.mark.parametrize("which,L", [("heisenberg_kitaev", 2), ("heisenberg_kitaev", 3), ("compass", 3)])
@pytest.mark.parametrize("lam", [0.05, 1.1])
def test_xyz_first_rhs_closed_form_bond_dependent(oracle_lib, which, L, lam):
    """The closed form of the first right-hand side (as above) for couplings
    that depend on the bond direction (Heisenberg-Kitaev honeycomb, J = 0.7,
    K = -1.3; square compass model): g and the lattice sum taken bond by bond
    from the model's interaction list by brute force over a cluster."""
    m = W.model_heisenberg_kitaev(0.7, -1.3) if which == "heisenberg_kitaev" else W.model_compass(0.9, -0.4)
    mesh = W.log_mesh(0.005, 50.0, 5)
    o = oracle_lib.Oracle(m, L, mesh)
    assert o.nc == 4
    d = o.rhs(lam, o.initial_state())
    sig, gx, gy, gz, gd = o.split(d)
    assert np.all(sig == 0.0)
    J = _coupling_by_bonds(m)
    cell = m.cell
    got = (gx, gy, gz)
    err = 0.0
    reach = L + 2
    cluster = [cell.position((d0, d1, 0), b) for d0 in range(-reach, reach + 1)
               for d1 in range(-reach, reach + 1) for b in range(cell.n_basis)]
    for b in range(o.lat.nb):
        rb = o.lat.basis_pos[b]
        for k in range(o.lat.nsites[b]):
            rk = o.lat.site_pos[b, k]
            g = J(rb, rk) / 4.0
            sgg = sum(J(rb, rj) * J(rj, rk) for rj in cluster) / 16.0
            for a in range(o.nf):
                for c in range(a + 1):
                    su = a * (a + 1) // 2 + c
                    for t in range(o.nf):
                        hs, hu, ht = _h(mesh[a], lam), _h(mesh[c], lam), _h(mesh[t], lam)
                        for mu in range(3):
                            nb_, nc_ = (mu + 1) % 3, (mu + 2) % 3
                            e = (-2.0 * g[nb_] * g[nc_] * (hs + hu) + 2.0 * ht * sgg[mu]) / (math.pi * lam)
                            err = max(err, abs(got[mu][b, su, t, k] - e))
                        ed = float(g @ g) / (math.pi * lam) * (hs - hu)
                        err = max(err, abs(gd[b, su, t, k] - ed))
    scale = max(np.abs(d).max(), 1.0)
    assert err <= 1e-14 * scale, (err, scale)
