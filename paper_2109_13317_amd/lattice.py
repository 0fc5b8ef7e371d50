"""Symmetry-reduced lattice tables for the flow library (Sec. 4.1).

This is the input front end of the library: it turns a unit cell, a coupling
model and a truncation range into the integer tables that the C-ABI
``pffrg_create`` consumes.  It runs once per lattice on the host; none of the
flow arithmetic happens here.

Construction (Sec. 4.1):
  * reference site i_ref = basis site 0 of cell 0;
  * lattice symmetries are Euclidean isometries x -> O x + v that map the
    lattice to itself, bonds to bonds and couplings to equal couplings (for
    XYZ models equal (Jx, Jy, Jz), for general models equal matrices on the
    directed bond; spin components are not permuted or rotated); they
    are found by mapping the nearest-neighbour bond vectors of one site onto
    those of another and validating the candidate on the unit cell;
  * for every basis site b one symmetry T_b with T_b(r_b) = r_ref, so any
    pair (i1, i2) maps to (i_ref, T(i2)) (Eq. 33);
  * sites within bond distance L of i_ref (Eq. 34) split into orbits of the
    stabiliser of i_ref (Eq. 35 without spin permutations, which SU(2) does
    not need); each orbit is one reduced pair, pair 0 is on-site;
  * tabulated lattice sums: for output pair p = (i_ref, j_p), every site k
    within range of both ends contributes Gamma_{i_ref k} Gamma_{k j_p}; k maps
    to pair ka and (k, j_p) maps, via T_k, to pair kb.  Equal (ka, kb) are
    merged with a multiplicity.

With ``spin_permutations=True`` (XYZ and general models, Sec. 4.1) a
symmetry is a lattice isometry together with a global spin transformation W,
a signed permutation of (x, y, z) with det W = +1 (a permutation with the
signs that make it a rotation: the flow equations are covariant under
rotations of the spin axes, not under reflections); it must map every
directed bond's matrix M to W^T M W (XYZ: (Jx, Jy, Jz) permuted, the signs
squaring away).  The vertex of the mapped pair then equals W^T Gamma W (the
density index untouched), so every pair exchange, lattice-sum factor and
chi site carries a rotation: Gamma_{i1 i2} = W Gamma_{i_ref j_q} W^T.
"""

from __future__ import annotations

from collections import deque
from dataclasses import dataclass
import itertools

import numpy as np

EPS = 1e-5      # real-space precision of the symmetry search (Sec. 4.1)


@dataclass
class LatticeTables:
    """Everything ``pffrg_create`` needs about the lattice, as flat arrays."""
    n_pairs: int
    swap: np.ndarray            # int32 [n_pairs]
    mult: np.ndarray            # int32 [n_pairs]
    rpa_off: np.ndarray         # int32 [n_pairs+1]
    rpa_ka: np.ndarray          # int32 [n_terms]
    rpa_kb: np.ndarray          # int32 [n_terms]
    rpa_cnt: np.ndarray         # int32 [n_terms]
    coupling: np.ndarray        # float64 [n_pairs], J of the bond (i_ref, j_p); XYZ: [n_pairs, 3];
                                # general: [n_pairs, 3, 3], M of S_ref . M . S_j
    n_basis: int
    n_sites_total: int
    site_pair: np.ndarray       # int32 [n_basis, n_sites_total]
    site_pos: np.ndarray        # float64 [n_basis, n_sites_total, 3]
    basis_pos: np.ndarray       # float64 [n_basis, 3]
    pair_rep: np.ndarray        # int32 [n_pairs, 4]: (cell0, cell1, cell2, basis)
    stabiliser_order: int
    # spin rotations (only with spin_permutations): rot[0] is the identity;
    # Gamma_{i1 i2} = W Gamma_q W^T with W = rot[id]
    rot: np.ndarray | None = None          # int32 [n_rot, 3, 3] signed permutation matrices
    swap_rot: np.ndarray | None = None     # int32 [n_pairs]: Gamma_{j_p i_ref} = W Gamma_{swap[p]} W^T
    rpa_rot_a: np.ndarray | None = None    # int32 [n_terms]: Gamma_{i_ref k} = W Gamma_{ka} W^T
    rpa_rot_b: np.ndarray | None = None    # int32 [n_terms]: Gamma_{k j_p} = W Gamma_{kb} W^T
    site_rot: np.ndarray | None = None     # int32 [n_basis, n_sites_total]: rotation of site_pair

    @property
    def n_terms(self) -> int:
        return int(self.rpa_off[-1])


class _Lattice:
    def __init__(self, cell, interactions, params):
        self.A = np.asarray(cell.primitives, dtype=np.float64)
        self.Ainv = np.linalg.inv(self.A)
        self.basis = np.asarray(cell.basis, dtype=np.float64)
        self.nb = len(self.basis)
        self.bonds = set()
        self.nbrs = [[] for _ in range(self.nb)]
        for (f, t, d0, d1, d2) in cell.bonds:
            d = (d0, d1, d2)
            self.bonds.add((f, t, d))
            self.bonds.add((t, f, (-d0, -d1, -d2)))
            self.nbrs[f].append((d, t))
            self.nbrs[t].append(((-d0, -d1, -d2), f))
        # couplings per directed bond: a number (Heisenberg), (Jx, Jy, Jz)
        # (XYZ) or a 3x3 matrix M of the term S_from . M . S_to (general
        # models; there numbers and triples become J 1 and diag(Jx, Jy, Jz),
        # and the reversed bond carries M^T)
        dims = {np.ndim(v) for v in params.values()}
        self.mat = 2 in dims
        self.vec = not self.mat and 1 in dims
        self.zero = np.zeros((3, 3)) if self.mat else (np.zeros(3) if self.vec else 0.0)
        self.J = {}
        for (pname, f, t, d0, d1, d2) in interactions:
            if self.mat:
                val = np.asarray(params.get(pname, self.zero), dtype=np.float64)
                if val.ndim < 2:
                    val = np.diag(np.broadcast_to(val, (3,)).astype(np.float64))
                rev = val.T
            elif self.vec:
                val = rev = np.asarray(params.get(pname, self.zero), dtype=np.float64)
            else:
                val = rev = float(params.get(pname, 0.0))
            for key, v in (((f, t, (d0, d1, d2)), val), ((t, f, (-d0, -d1, -d2)), rev)):
                self.J[key] = self.J.get(key, self.zero) + v

    def pos(self, cell, b):
        return np.asarray(cell, dtype=np.float64) @ self.A + self.basis[b]

    def locate(self, p):
        """(cell, basis) of the lattice site at position p, or None."""
        for b in range(self.nb):
            f = (p - self.basis[b]) @ self.Ainv
            r = np.rint(f)
            if np.abs(f - r).max() < EPS:
                return (int(r[0]), int(r[1]), int(r[2])), b
        return None

    def coupling(self, c1, b1, c2, b2):
        d = (c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2])
        return self.J.get((b1, b2, d), self.zero)

    def bonded(self, c1, b1, c2, b2):
        d = (c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2])
        return (b1, b2, d) in self.bonds

    def ball(self, b, L):
        """Sites within bond distance L of (cell 0, b), BFS order, with distances."""
        start = ((0, 0, 0), b)
        dist = {start: 0}
        order = [start]
        q = deque([start])
        while q:
            node = q.popleft()
            if dist[node] == L:
                continue
            (c, bb) = node
            for (d, b2) in self.nbrs[bb]:
                nxt = ((c[0] + d[0], c[1] + d[1], c[2] + d[2]), b2)
                if nxt not in dist:
                    dist[nxt] = dist[node] + 1
                    order.append(nxt)
                    q.append(nxt)
        return order, dist


class _Iso:
    """x -> O x + v, with the spin transformation R (3x3, identity unless
    spin permutations are searched)."""

    def __init__(self, O, v, R=None):
        self.O, self.v = O, v
        self.R = np.eye(3) if R is None else R

    def apply(self, lat, site):
        c, b = site
        return lat.locate(self.O @ lat.pos(c, b) + self.v)


def _frame(vecs):
    """Three independent vectors from a neighbour-vector list (normal added
    for planar stars); returns (indices, matrix) or raises."""
    vecs = [np.asarray(v) for v in vecs]
    for i, j in itertools.permutations(range(len(vecs)), 2):
        n = np.cross(vecs[i], vecs[j])
        if np.linalg.norm(n) < EPS:
            continue
        for k in range(len(vecs)):
            if abs(np.dot(n, vecs[k])) > EPS:
                return (i, j, k), np.array([vecs[i], vecs[j], vecs[k]])
        return (i, j, -1), np.array([vecs[i], vecs[j], n / np.linalg.norm(n)])
    raise ValueError("bond star does not span two dimensions")


def _proper_signed_permutations():
    """The 24 signed permutation matrices with determinant +1, identity first."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            W = np.zeros((3, 3))
            for r in range(3):
                W[r, perm[r]] = signs[r]
            if round(np.linalg.det(W)) == 1:
                out.append(W)
    out.sort(key=lambda W: not np.array_equal(W, np.eye(3)))
    return out


def _symmetries_onto(lat, b_from, b_to, spins=(None,)):
    """All lattice symmetries g with g(r_{b_from}) = r_{b_to} (both in cell 0),
    each with every spin transformation in ``spins`` under which it is one."""
    src = [lat.pos(d, t) - lat.pos((0, 0, 0), b_from) for (d, t) in lat.nbrs[b_from]]
    dst = [lat.pos(d, t) - lat.pos((0, 0, 0), b_to) for (d, t) in lat.nbrs[b_to]]
    (i, j, k), X = _frame(src)
    r_from, r_to = lat.pos((0, 0, 0), b_from), lat.pos((0, 0, 0), b_to)
    out = []
    cand_k = range(len(dst)) if k >= 0 else (None,)
    for ii, jj in itertools.permutations(range(len(dst)), 2):
        for kk in cand_k:
            rows = [dst[ii], dst[jj]]
            if kk is None:
                n = np.cross(dst[ii], dst[jj])
                if np.linalg.norm(n) < EPS:
                    continue
                n = n / np.linalg.norm(n)
                choices = [rows + [n], rows + [-n]]
            else:
                if kk in (ii, jj):
                    continue
                choices = [rows + [dst[kk]]]
            for Yr in choices:
                Y = np.array(Yr)
                try:
                    O = np.linalg.solve(X, Y).T        # O X^T = Y^T
                except np.linalg.LinAlgError:
                    continue
                if np.abs(O.T @ O - np.eye(3)).max() > EPS:
                    continue
                for R in spins:
                    g = _Iso(O, r_to - O @ r_from, R)
                    if any(np.abs(O - h.O).max() < EPS and np.abs(g.R - h.R).max() < EPS for h in out):
                        continue
                    if _valid(lat, g):
                        out.append(g)
    return out


def _valid(lat, g):
    """g maps lattice translations to translations, basis sites to sites,
    and every bond / coupling of the unit cell to an equal one."""
    for a in lat.A:
        f = (g.O @ a) @ lat.Ainv
        if np.abs(f - np.rint(f)).max() > EPS:
            return False
    img = {}
    for b in range(lat.nb):
        s = g.apply(lat, ((0, 0, 0), b))
        if s is None:
            return False
        img[b] = s
    keys = set(lat.bonds) | set(lat.J)
    for (b1, b2, d) in keys:
        s1 = img[b1]
        s2 = g.apply(lat, (d, b2))
        if s2 is None:
            return False
        if lat.bonded(s1[0], s1[1], s2[0], s2[1]) != ((b1, b2, d) in lat.bonds):
            return False
        want = lat.J.get((b1, b2, d), lat.zero)
        if lat.mat:
            want = g.R.T @ want @ g.R           # J_{g i, g j} = R^T J_ij R
        elif lat.vec:
            want = np.diag(g.R.T @ np.diag(want) @ g.R)    # (Jx, Jy, Jz) permuted
        if np.max(np.abs(lat.coupling(s1[0], s1[1], s2[0], s2[1]) - want)) > 1e-12:
            return False
    return True


def build_tables(model, L: int, spin_permutations: bool = False) -> LatticeTables:
    """Reduced pair tables for ``model`` (a ``workloads.Model``) at range L;
    spin_permutations: also search joint lattice and spin transformations
    (XYZ and general models)."""
    lat = _Lattice(model.cell, model.interactions, model.params)
    L = int(L)
    if spin_permutations and not (lat.mat or lat.vec):
        raise ValueError("spin permutations need an XYZ or a general model (SU(2) couplings are invariant)")
    spins = _proper_signed_permutations() if spin_permutations else (None,)
    stab = _symmetries_onto(lat, 0, 0, spins)
    to_ref = []
    for b in range(lat.nb):
        gs = _symmetries_onto(lat, b, 0, spins)
        if not gs:
            raise ValueError(f"basis site {b} is not equivalent to the reference site")
        to_ref.append(gs[0])
    rots = [np.eye(3)]

    def rot_id(W):
        for i, V in enumerate(rots):
            if np.abs(V - W).max() < 0.5:
                return i
        rots.append(np.rint(W))
        return len(rots) - 1

    ball0, dist0 = lat.ball(0, L)
    in_ball = set(ball0)
    orbit_of = {}
    xrot = {}           # Gamma_{i_ref k} = X Gamma_{rep} X^T
    reps = []
    mult = []
    for site in ball0:
        if site in orbit_of:
            continue
        p = len(reps)
        reps.append(site)
        members = {site: np.eye(3)}
        for g in stab:
            im = g.apply(lat, site)
            if im not in members:
                members[im] = g.R.T      # Gamma_{ref, g r} = R^T Gamma_{ref, r} R
        for m, X in members.items():
            if m not in in_ball:
                raise RuntimeError("stabiliser does not preserve the truncation ball")
            orbit_of[m] = p
            xrot[m] = X
        mult.append(len(members))
    n_pairs = len(reps)

    def to_reference_rot(site_a, site_b):
        """(reduced pair, W) with Gamma_{a b} = W Gamma_pair W^T, or (-1, None) out of range."""
        (ca, ba) = site_a
        (cb, bb) = site_b
        shifted = ((cb[0] - ca[0], cb[1] - ca[1], cb[2] - ca[2]), bb)
        g = to_ref[ba]
        im = g.apply(lat, shifted)
        if im not in orbit_of:
            return -1, None
        return orbit_of[im], g.R @ xrot[im]      # Gamma_{a b} = R Gamma_{ref, g b} R^T

    def to_reference(site_a, site_b):
        """Reduced pair of (site_a, site_b), or -1 if out of range."""
        return to_reference_rot(site_a, site_b)[0]

    sw = [to_reference_rot(r, ((0, 0, 0), 0)) for r in reps]
    swap = np.array([q for q, _ in sw], dtype=np.int32)
    if (swap < 0).any():
        raise RuntimeError("pair swap left the truncation range")
    swap_rot = np.array([rot_id(W) for _, W in sw], dtype=np.int32)

    off = [0]
    ka_l, kb_l, cnt_l, ra_l, rb_l = [], [], [], [], []
    for p, rep in enumerate(reps):
        terms = {}
        for k in ball0:
            kb, Wb = to_reference_rot(k, rep)
            if kb < 0:
                continue
            key = (orbit_of[k], kb, rot_id(xrot[k]), rot_id(Wb))
            terms[key] = terms.get(key, 0) + 1
        for (a, b, ra, rb), n in sorted(terms.items()):
            ka_l.append(a); kb_l.append(b); cnt_l.append(n); ra_l.append(ra); rb_l.append(rb)
        off.append(len(ka_l))

    coupling = np.array([lat.coupling((0, 0, 0), 0, r[0], r[1]) for r in reps])

    balls = [lat.ball(b, L)[0] for b in range(lat.nb)]
    ntot = max(len(bl) for bl in balls)
    site_pair = np.full((lat.nb, ntot), -1, dtype=np.int32)
    site_rot = np.zeros((lat.nb, ntot), dtype=np.int32)
    site_pos = np.zeros((lat.nb, ntot, 3))
    for b, bl in enumerate(balls):
        for k, site in enumerate(bl):
            q, W = to_reference_rot(((0, 0, 0), b), site)
            site_pair[b, k] = q
            if q >= 0:
                site_rot[b, k] = rot_id(W)
            site_pos[b, k] = lat.pos(*site)
    if (site_pair[site_pair != -1] < 0).any():
        raise RuntimeError("site map incomplete")

    return LatticeTables(
        n_pairs=n_pairs, swap=swap, mult=np.array(mult, dtype=np.int32),
        rpa_off=np.array(off, dtype=np.int32), rpa_ka=np.array(ka_l, dtype=np.int32),
        rpa_kb=np.array(kb_l, dtype=np.int32), rpa_cnt=np.array(cnt_l, dtype=np.int32),
        coupling=coupling, n_basis=lat.nb, n_sites_total=ntot, site_pair=site_pair,
        site_pos=site_pos, basis_pos=lat.basis.copy(),
        pair_rep=np.array([[r[0][0], r[0][1], r[0][2], r[1]] for r in reps], dtype=np.int32),
        stabiliser_order=len(stab),
        **(dict(rot=np.array(rots, dtype=np.int32), swap_rot=swap_rot,
                rpa_rot_a=np.array(ra_l, dtype=np.int32), rpa_rot_b=np.array(rb_l, dtype=np.int32),
                site_rot=site_rot) if spin_permutations else {}))


@dataclass
class LatticeDescription:
    """The lattice spin model as built, for checking it by eye or by script
    (the lattice description output of Sec. 5, "Output data")."""
    positions: np.ndarray       # float64 [n_sites, 3], site id = row
    parametrized: np.ndarray    # bool [n_sites]: the site represents a reduced pair
    bonds: list                 # [(from id, to id)], once per unit-cell bond
    interactions: list          # [(from id, to id, J)], Heisenberg: J times the 3x3 identity


def describe(model, L: int) -> LatticeDescription:
    """Sites within bond distance L of the reference site (breadth-first
    order, id 0 the reference site), the lattice bonds and the nonzero
    couplings between them, each listed once in the orientation of the unit
    cell or model that defines it, and which sites are parametrized: the
    representatives of the reduced pairs that ``build_tables`` keeps."""
    lat = _Lattice(model.cell, model.interactions, model.params)
    sites, _ = lat.ball(0, int(L))
    ids = {s: i for i, s in enumerate(sites)}
    reps = {((int(r[0]), int(r[1]), int(r[2])), int(r[3])) for r in build_tables(model, L).pair_rep}

    def links(defs):
        out = {}
        for (c, b) in sites:
            for (val, f, t, d0, d1, d2) in defs:
                if f != b:
                    continue
                j = ids.get(((c[0] + d0, c[1] + d1, c[2] + d2), t))
                if j is not None:
                    out[(ids[(c, b)], j)] = out.get((ids[(c, b)], j), 0.0) + val
        return out

    bonds = sorted(links([(1.0,) + tuple(bd) for bd in model.cell.bonds]))
    # a coupling is a number (Heisenberg), (Jx, Jy, Jz) (XYZ) or a 3x3 matrix
    def value(p):
        if lat.mat:
            v = np.asarray(model.params.get(p, lat.zero), dtype=np.float64)
            return v if v.ndim == 2 else np.diag(np.broadcast_to(v, (3,)).astype(np.float64))
        if lat.vec:
            return np.asarray(model.params.get(p, lat.zero), dtype=np.float64)
        return float(model.params.get(p, 0.0))
    coup = links([(value(p), f, t, d0, d1, d2) for (p, f, t, d0, d1, d2) in model.interactions])
    return LatticeDescription(
        positions=np.array([lat.pos(*s) for s in sites]),
        parametrized=np.array([s in reps for s in sites]),
        bonds=bonds,
        interactions=[(i, j, v) for (i, j), v in sorted(coup.items()) if np.any(np.asarray(v) != 0.0)])
