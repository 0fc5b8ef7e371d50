"""Pins of the oracle's general (TRI) form: couplings S_i . M_ij . S_j with any
real 3x3 matrices (Sec. 2), all sixteen vertex components (Sec. 3, Eq. 16),
held as real numbers r with Gamma = r where xi(mu) xi(nu) = 1 and Gamma = i r
where it is -1 (Eq. 18).

  XYZ limit               diagonal couplings and a diagonal state: the
                          sixteen-strain flow equals the four-strain XYZ flow
                          (whose hand-contracted coefficients have their own
                          pins) and no off-diagonal component flows
  literal evaluation      the C oracle against the explicit spin-index
                          equations of oracle/literal.py on random states:
                          self-energy, every vertex component and chi; the
                          parts the real representation drops vanish
  first right-hand side   closed form at Sigma = 0, Gamma = J/4 in two-spin
                          operator language (Kronecker products, a partial
                          transpose, a 4x4 matrix product for the lattice sum),
                          derived by hand from Eq. 24 independently of the
                          index contractions of the oracle
  spin rotations          a global rotation R of the spin axes maps the flow
                          of a rotated state onto the rotated flow, and chi
                          onto R chi R^T: the flow equations are covariant
  J = 0                   every right-hand side vanishes
"""

import math

import numpy as np
import pytest

import workloads as W
from workloads import Model

XI = np.array([1.0, -1.0, -1.0, -1.0])
XIXI = np.outer(XI, XI)
SIG = np.array([[[1, 0], [0, 1]], [[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]],
               dtype=np.complex128)


def _h(v, lam):
    return 1.0 / (v + lam) - (1.0 / (v - lam) if v > 2.0 * lam else 0.0)


def _tri_model(lattice, **shells):
    """A general model on the Heisenberg bonds of ``lattice``: 3x3 matrix per shell."""
    base = W.model(lattice)
    params = {k: np.zeros((3, 3)) for k in base.params}
    for k, v in shells.items():
        params[k] = np.asarray(v, dtype=float)
    return Model(f"{lattice}-tri", base.cell, base.interactions, params)


def _dm(d, jd=1.0, gamma=None):
    """J on the diagonal plus a Dzyaloshinskii-Moriya vector d (M^{ab} = eps_{abc} d_c)
    plus an optional symmetric off-diagonal part."""
    m = jd * np.eye(3)
    m[0, 1], m[1, 0] = d[2], -d[2]
    m[1, 2], m[2, 1] = d[0], -d[0]
    m[2, 0], m[0, 2] = d[1], -d[1]
    if gamma is not None:
        m = m + np.asarray(gamma, dtype=float)
    return m


M_SQ = _dm((0.1, -0.2, 0.35), 1.0, [[0.0, 0.15, 0.0], [0.15, -0.2, 0.3], [0.0, 0.3, 0.1]])
M_SQ2 = _dm((0.0, 0.0, -0.15), 0.3, [[0.05, 0.0, 0.1], [0.0, 0.0, 0.0], [0.1, 0.0, -0.1]])


def _random_tri_state(o, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    x = o.initial_state()
    parts = o.split(x)
    parts[0][:] = -np.abs(rng.normal(0, scale, o.nf))
    for q in range(16):
        parts[1 + q][...] = rng.normal(0, scale, parts[1 + q].shape)
    for a in range(o.nf):                     # Gamma^{mu 0}(s, t, s) = 0 by the s <-> u relation
        for m in range(4):
            parts[1 + 4 * m][:, a * (a + 1) // 2 + a] = 0.0
    return x


def test_tri_layout_and_initial_state(oracle_lib):
    o = oracle_lib.Oracle(_tri_model("square", j1=M_SQ), 2, W.log_mesh(0.01, 10.0, 4))
    assert o.symmetry == "tri" and o.nc == 16
    x = o.initial_state()
    parts = o.split(x)
    assert np.all(parts[0] == 0.0)
    lat = o.lat
    for k in range(lat.nsites[0]):
        J = lat.coupling[0, k]
        for m in range(4):
            for n in range(4):
                want = J[m - 1, n - 1] / 4.0 if m and n else 0.0
                assert np.all(parts[1 + 4 * m + n][0, :, :, k] == want)
    # a bond and its reverse carry M and M^T
    k1 = lat.index(0, (1, 0, 0), 0)
    km = lat.index(0, (-1, 0, 0), 0)
    assert np.array_equal(lat.coupling[0, km], lat.coupling[0, k1].T)
    assert np.array_equal(lat.coupling[0, k1], M_SQ) or np.array_equal(lat.coupling[0, km], M_SQ)


@pytest.mark.parametrize("L", [1, 2])
def test_tri_reduces_to_xyz(oracle_lib, L):
    """Bond-dependent diagonal couplings (Heisenberg-Kitaev honeycomb) and a
    diagonal state: the TRI flow equals the XYZ flow strain by strain, no
    off-diagonal component flows, and chi agrees."""
    mx = W.model_heisenberg_kitaev(0.8, -1.1)
    mt = Model("hk-tri", mx.cell, mx.interactions, {k: np.diag(v) for k, v in mx.params.items()})
    mesh = W.log_mesh(0.02, 20.0, 5)
    ox = oracle_lib.Oracle(mx, L, mesh)
    ot = oracle_lib.Oracle(mt, L, mesh)
    rng = np.random.default_rng(11)
    xx = ox.initial_state()
    px = ox.split(xx)
    px[0][:] = -np.abs(rng.normal(0, 0.3, ox.nf))
    for c in range(4):
        px[1 + c][...] += rng.normal(0, 0.3, px[1 + c].shape)
    for a in range(ox.nf):
        px[4][:, a * (a + 1) // 2 + a] = 0.0
    pairs = ((0, 5), (1, 10), (2, 15), (3, 0))          # (XYZ strain, TRI strain)

    def embed(x4):
        x16 = np.zeros(ot.size)
        p4, p16 = ox.split(x4), ot.split(x16)
        p16[0][:] = p4[0]
        for c, q in pairs:
            p16[1 + q][...] = p4[1 + c]
        return x16

    assert np.array_equal(ot.initial_state(), embed(ox.initial_state()))
    xt = embed(xx)
    for lam in (0.03, 0.6, 5.0):
        d4, d16 = ox.rhs(lam, xx), ot.rhs(lam, xt)
        scale = np.abs(d4).max()
        assert np.abs(d16 - embed(d4)).max() <= 1e-13 * scale, lam
        c4 = ox.chi_comps(lam, xx)
        re, im = ot.chi_tri(lam, xt)
        cs = np.abs(c4).max()
        for c, mu in ((0, 1), (1, 2), (2, 3), (3, 0)):
            assert np.abs(re[mu, mu] - c4[c]).max() <= 1e-13 * cs
        off = max(np.abs(re[a, b]).max() for a in range(4) for b in range(4) if a != b)
        assert off <= 1e-13 * cs and np.abs(im).max() <= 1e-13 * cs


@pytest.mark.parametrize("lam", [0.04, 0.55, "mesh"])
def test_tri_c_oracle_matches_literal_spin_evaluation(oracle_lib, lam):
    from oracle.literal import LiteralFlow
    o = oracle_lib.Oracle(_tri_model("square", j1=M_SQ, j2=M_SQ2), 1, W.log_mesh(0.05, 5.0, 4))
    if lam == "mesh":
        lam = float(o.mesh[2])
    x = _random_tri_state(o, 23)
    lf = LiteralFlow(o)
    ds_c = o.sigma_rhs(lam, x)
    ds_a = lf.sigma_rhs(lam, x)
    # the real representation keeps the imaginary (Eq. 15) part of dSigma
    assert np.abs(ds_c - ds_a.imag).max() <= 1e-14 * max(1.0, np.abs(ds_c).max())
    full = o.rhs(lam, x)
    parts = o.split(full)
    scale = max(np.abs(full).max(), 1.0)
    dropped = 0.0
    for k in range(o.lat.nsites[0]):
        for a in range(o.nf):
            for c in range(a + 1):
                for t in range(o.nf):
                    r = lf.vertex_rhs(lam, x, ds_c, 0, k, a, t, c)
                    su = a * (a + 1) // 2 + c
                    keep = np.where(XIXI > 0, r.real, r.imag)
                    drop = np.where(XIXI > 0, r.imag, r.real)
                    got = np.array([parts[1 + q][0, su, t, k] for q in range(16)]).reshape(4, 4)
                    assert np.abs(got - keep).max() <= 1e-13 * scale
                    dropped = max(dropped, np.abs(drop).max())
    # Eq. 18: every component comes out real resp. imaginary as its xi xi says
    assert dropped <= 1e-13 * scale
    re, im = o.chi_tri(lam, x)
    for k in range(o.lat.nsites[0]):
        for mu in range(4):
            v = lf.chi(lam, x, 0, k, mu)
            assert abs(re[mu, mu, 0, k] - v.real) <= 1e-13 and abs(im[mu, mu, 0, k] - v.imag) <= 1e-13


def _coupling_by_bonds(model):
    """M(r_i, r_j): the 3x3 coupling of the term S_i . M . S_j summed over
    every listed interaction (param, b0, b1, d) joining sublattice b0 in any
    cell R with sublattice b1 in cell R + d; the reverse direction gets M^T."""
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
        tot = np.zeros((3, 3))
        for (name, b0, b1, d0, d1, d2) in model.interactions:
            v = np.asarray(model.params[name], dtype=float)
            dr = np.array([d0, d1, d2], dtype=float) @ P + B[b1] - B[b0]
            if bi == b0 and bj == b1 and np.abs(rj - ri - dr).max() < 1e-9:
                tot += v
            if bi == b1 and bj == b0 and np.abs(ri - rj - dr).max() < 1e-9:
                tot += v.T
        return tot
    return J


def _two_spin(G):
    """V = sum Gamma^{mu nu} sigma^mu (x) sigma^nu (Eq. 25) from the complex 4x4 Gamma."""
    return sum(G[m, n] * np.kron(SIG[m], SIG[n]) for m in range(4) for n in range(4))


def _basis(V):
    """Gamma^{mu nu} = tr(V sigma^mu (x) sigma^nu) / 4."""
    return np.array([[np.trace(V @ np.kron(SIG[m], SIG[n])) / 4.0 for n in range(4)] for m in range(4)])


def _t1(V):
    """Partial transpose on the first spin of a two-spin operator."""
    return V.reshape(2, 2, 2, 2).transpose(2, 1, 0, 3).reshape(4, 4)


@pytest.mark.parametrize("lattice,shells,L", [
    ("square", dict(j1=M_SQ, j2=M_SQ2), 2),
    ("honeycomb", dict(j1=_dm((0.0, 0.0, 0.4), 0.9, [[0, 0.3, 0], [0.3, 0, 0], [0, 0, 0]]),
                       j2=_dm((0.2, 0.0, -0.1), 0.2)), 2),
])
@pytest.mark.parametrize("lam", [0.037, 0.9])
def test_tri_first_rhs_closed_form(oracle_lib, lattice, shells, L, lam):
    """At Sigma = 0 and Gamma^{ab} = J^{ab}/4 (spin indices; every component
    with a density index zero) the flow has no Katanin part and the bubbles
    are B_s = h(s)/(pi lam), B_t = B_u = -h/(pi lam).  In two-spin operator
    language, with V = sum G^{mu nu} sigma^mu (x) sigma^nu:
      s channel  V V                      (legs (1'2';34)(34;12): operator product)
      u channel  T1(T1(V) T1(V))          (the first spin's product reversed)
      t channel  -2 sum_j G_{i1 j} G_{j i2} (spin traces over the inner legs
                 leave a matrix product of the 4x4 coefficient matrices);
    the on-site vertex corrections vanish (no on-site coupling).  So
      dG = [h(s) P(V V) - h(u) P(T1(T1 V T1 V)) + 2 h(t) sum_j G G] / (pi lam)."""
    m = _tri_model(lattice, **shells)
    mesh = W.log_mesh(0.005, 50.0, 5)
    o = oracle_lib.Oracle(m, L, mesh)
    d = o.rhs(lam, o.initial_state())
    parts = o.split(d)
    assert np.all(parts[0] == 0.0)
    J = _coupling_by_bonds(m)
    cell = m.cell
    reach = L + 2
    cluster = [cell.position((d0, d1, 0), b) for d0 in range(-reach, reach + 1)
               for d1 in range(-reach, reach + 1) for b in range(cell.n_basis)]

    def G_of(ri, rj):
        G = np.zeros((4, 4), dtype=np.complex128)
        G[1:, 1:] = J(ri, rj) / 4.0
        return G

    err = 0.0
    imag_like = 0.0
    for b in range(o.lat.nb):
        rb = o.lat.basis_pos[b]
        for k in range(o.lat.nsites[b]):
            rk = o.lat.site_pos[b, k]
            G = G_of(rb, rk)
            V = _two_spin(G)
            Ps = _basis(V @ V)
            Pu = _basis(_t1(_t1(V) @ _t1(V)))
            Pt = 2.0 * sum(G_of(rb, rj) @ G_of(rj, rk) for rj in cluster)
            for a in range(o.nf):
                for c in range(a + 1):
                    su = a * (a + 1) // 2 + c
                    for t in range(o.nf):
                        e = (_h(mesh[a], lam) * Ps - _h(mesh[c], lam) * Pu + _h(mesh[t], lam) * Pt) / (math.pi * lam)
                        keep = np.where(XIXI > 0, e.real, e.imag)
                        imag_like = max(imag_like, np.abs(np.where(XIXI > 0, e.imag, e.real)).max())
                        got = np.array([parts[1 + q][b, su, t, k] for q in range(16)]).reshape(4, 4)
                        err = max(err, np.abs(got - keep).max())
    scale = max(np.abs(d).max(), 1.0)
    assert imag_like <= 1e-15 * scale
    assert err <= 1e-14 * scale, (err, scale)
    # the off-diagonal and density-spin components do flow here
    assert max(np.abs(parts[1 + q]).max() for q in (1, 2, 3, 4, 8, 12, 6, 7, 9)) > 1e-3 * scale


def _rotation(seed):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _rotate_state(o, x, R):
    """Gamma^{mu nu} -> R4 Gamma R4^T with R4 = diag(1, R) on every element
    (the spin indices rotate, the density index stays); sigma unchanged."""
    R4 = np.eye(4)
    R4[1:, 1:] = R
    y = x.copy()
    px, py = o.split(x), o.split(y)
    G = np.stack([px[1 + q] for q in range(16)], axis=-1)
    G = G.reshape(G.shape[:-1] + (4, 4))
    Gr = np.einsum("ma,...ab,nb->...mn", R4, G, R4)
    for q in range(16):
        py[1 + q][...] = Gr[..., q // 4, q % 4]
    return y


@pytest.mark.parametrize("lam", [0.05, 0.8])
def test_tri_spin_rotation_covariance(oracle_lib, lam):
    """Rotating the spin axes of the state by R (an element of SO(3)) rotates
    the flow: rhs(R x) = R rhs(x), the self-energy flow is unchanged, and
    chi^{ab} -> R chi R^T.  The rotation mixes the real (spin-spin, density-
    density) components among themselves and the imaginary (density-spin)
    ones among themselves, so the real representation is kept."""
    o = oracle_lib.Oracle(_tri_model("honeycomb", j1=M_SQ, j2=M_SQ2), 2, W.log_mesh(0.03, 8.0, 4))
    x = _random_tri_state(o, 31)
    R = _rotation(7)
    xr = _rotate_state(o, x, R)
    d, dr = o.rhs(lam, x), o.rhs(lam, xr)
    want = _rotate_state(o, d, R)
    scale = np.abs(d).max()
    assert np.abs(dr - want).max() <= 1e-13 * scale
    re, im = o.chi_tri(lam, x)
    rer, imr = o.chi_tri(lam, xr)
    R4 = np.eye(4)
    R4[1:, 1:] = R
    for arr, arr_r in ((re, rer), (im, imr)):
        rot = np.einsum("ma,ab...,nb->mn...", R4, arr, R4)
        assert np.abs(arr_r - rot).max() <= 1e-13 * np.abs(re).max()


def test_tri_zero_coupling_is_a_fixed_point(oracle_lib):
    o = oracle_lib.Oracle(_tri_model("square", j1=np.zeros((3, 3))), 2, W.log_mesh(0.005, 50.0, 5))
    x = o.initial_state()
    x[: o.nf] = -np.linspace(0.1, 0.4, o.nf)
    for lam in (0.01, 0.5, 20.0):
        assert np.all(o.rhs(lam, x) == 0.0)
