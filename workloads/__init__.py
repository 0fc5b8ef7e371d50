"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds *inputs only*: lattice unit cells, coupling definitions,
frequency meshes, cutoff schedules, the five benchmark workloads and seeded
random flow states.  It contains none of the pf-FRG arithmetic (no
propagators, no flow equations, no symmetry reduction), so that the oracle and
the GPU library can both consume it without sharing any method code.

Unit cells follow the resource-file format of the paper (Sec. 5.2, "Definition
of lattice graphs": three primitive vectors, basis sites, and bonds given as
(from, to, da0, da1, da2)).  Couplings follow Sec. 5.3 ("Definition of spin
interactions"): each interaction joins a site of the home cell to a site given
by (da0, da1, da2, basis) and carries a named Heisenberg parameter.  Each
unordered bond of the infinite lattice appears exactly once per unit cell.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "UnitCell", "Model", "UNIT_CELLS", "unit_cell", "model", "model_xyz", "model_kitaev_gamma", "model_dm",
    "log_mesh", "exponential_schedule", "geometric_schedule",
    "Workload", "workload", "WORKLOAD_NAMES", "batch_scan_points",
    "random_state", "state_layout",
]


@dataclass(frozen=True)
class UnitCell:
    """A lattice unit cell embedded in three dimensions (Sec. 5.2)."""
    name: str
    primitives: np.ndarray          # (3, 3): rows are a0, a1, a2
    basis: np.ndarray               # (nb, 3) Cartesian basis-site positions
    bonds: tuple                    # ((from, to, da0, da1, da2), ...)

    @property
    def n_basis(self) -> int:
        return int(self.basis.shape[0])

    def position(self, cell, b) -> np.ndarray:
        cell = np.asarray(cell, dtype=np.float64)
        return cell @ self.primitives + self.basis[b]


def _bonds_by_distance(prims, basis, dist, tol=1e-6, reach=2):
    """Every bond of length ``dist`` once per unit cell, canonical orientation."""
    out = []
    nb = len(basis)
    rng = range(-reach, reach + 1)
    for b0 in range(nb):
        for d0 in rng:
            for d1 in rng:
                for d2 in rng:
                    for b1 in range(nb):
                        r = np.array([d0, d1, d2]) @ prims + basis[b1] - basis[b0]
                        if abs(np.linalg.norm(r) - dist) > tol:
                            continue
                        fwd = (b0, (d0, d1, d2), b1)
                        rev = (b1, (-d0, -d1, -d2), b0)
                        if fwd <= rev:
                            out.append((b0, b1, d0, d1, d2))
    return tuple(sorted(set(out)))


_S3 = math.sqrt(3.0)

UNIT_CELLS = {
    # Sec. 5.2, listing of unit cells: square lattice.
    "square": UnitCell(
        "square",
        np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]),
        np.array([[0.0, 0.0, 0.0]]),
        ((0, 0, 1, 0, 0), (0, 0, 0, 1, 0)),
    ),
    # Sec. 5.2, listing of unit cells: honeycomb lattice.
    "honeycomb": UnitCell(
        "honeycomb",
        np.array([[1.5, _S3 / 2, 0.0], [1.5, -_S3 / 2, 0.0], [0.0, 0.0, 1.0]]),
        np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]]),
        ((0, 1, 0, 0, 0), (1, 0, 1, 0, 0), (1, 0, 0, 1, 0)),
    ),
    # Sec. 6.1: simple cubic lattice.
    "cubic": UnitCell(
        "cubic",
        np.eye(3),
        np.array([[0.0, 0.0, 0.0]]),
        ((0, 0, 1, 0, 0), (0, 0, 0, 1, 0), (0, 0, 0, 0, 1)),
    ),
}

# Pyrochlore: fcc primitives with the four-site tetrahedral basis; bonds join
# nearest neighbours at distance sqrt(2)/4.
_PY_PRIMS = np.array([[0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
_PY_BASIS = np.array([[0.0, 0.0, 0.0], [0.0, 0.25, 0.25], [0.25, 0.0, 0.25], [0.25, 0.25, 0.0]])
UNIT_CELLS["pyrochlore"] = UnitCell(
    "pyrochlore", _PY_PRIMS, _PY_BASIS,
    _bonds_by_distance(_PY_PRIMS, _PY_BASIS, math.sqrt(2.0) / 4.0),
)


def unit_cell(name: str) -> UnitCell:
    return UNIT_CELLS[name]


@dataclass(frozen=True)
class Model:
    """Spin couplings on a unit cell (Sec. 5.3).

    ``interactions`` lists (param, b_from, b_to, da0, da1, da2); the value of
    each named parameter is in ``params``.  A number J is a Heisenberg
    coupling, J S_from . S_to; a triple (Jx, Jy, Jz) an XYZ coupling,
    Jx S^x S^x + Jy S^y S^y + Jz S^z S^z (Sec. 2); a 3x3 matrix M the general
    coupling S_from . M . S_to (Sec. 2, Sec. 5.3), which has a direction: the
    reversed bond carries M^T.  The Hamiltonian is the sum
    over every listed bond and all lattice translations, each unordered bond
    counted once.
    """
    name: str
    cell: UnitCell
    interactions: tuple
    params: dict = field(default_factory=dict)

    def with_params(self, **kw) -> "Model":
        p = dict(self.params)
        p.update(kw)
        return Model(self.name, self.cell, self.interactions, p)

    @property
    def symmetry(self) -> str:
        """'tri' when a coupling is a 3x3 matrix M (the term S_from . M . S_to,
        Sec. 5.3), 'xyz' when the couplings are (Jx, Jy, Jz) triples, else
        'su2'."""
        dims = {np.ndim(v) for v in self.params.values()}
        return "tri" if 2 in dims else ("xyz" if 1 in dims else "su2")


# Coupling shells by Euclidean distance: (parameter name, distance).
_SHELLS = {
    "square": (("j1", 1.0), ("j2", math.sqrt(2.0)), ("j3", 2.0)),
    "honeycomb": (("j1", 1.0), ("j2", _S3), ("j3", 2.0)),
    "cubic": (("j1", 1.0), ("j2", math.sqrt(2.0))),
    "pyrochlore": (("j1", math.sqrt(2.0) / 4.0),),
}


def model(lattice: str, **params) -> Model:
    """Heisenberg model on ``lattice`` with shell couplings j1, j2, ... ."""
    cell = UNIT_CELLS[lattice]
    inter = []
    for pname, dist in _SHELLS[lattice]:
        for (b0, b1, d0, d1, d2) in _bonds_by_distance(cell.primitives, cell.basis, dist):
            inter.append((pname, b0, b1, d0, d1, d2))
    full = {name: 0.0 for name, _ in _SHELLS[lattice]}
    full.update({k: float(v) for k, v in params.items()})
    unknown = set(params) - {n for n, _ in _SHELLS[lattice]}
    if unknown:
        raise ValueError(f"unknown couplings {sorted(unknown)} for {lattice}")
    return Model(f"{lattice}-heisenberg", cell, tuple(inter), full)


def model_xyz(lattice: str, **params) -> Model:
    """XYZ model on ``lattice`` with shell couplings j1=(Jx, Jy, Jz), ...
    (the same bonds as ``model``; unnamed shells are (0, 0, 0))."""
    base = model(lattice)
    full = {name: (0.0, 0.0, 0.0) for name in base.params}
    for k, v in params.items():
        if k not in full:
            raise ValueError(f"unknown coupling {k} for {lattice}")
        v = tuple(float(x) for x in v)
        if len(v) != 3:
            raise ValueError(f"{k}: an XYZ coupling is a triple (Jx, Jy, Jz)")
        full[k] = v
    return Model(f"{lattice}-xyz", base.cell, base.interactions, full)


def model_heisenberg_kitaev(J: float = 1.0, K: float = 0.0) -> Model:
    """Heisenberg-Kitaev model on the honeycomb lattice: J S_i . S_j + K S_i^g
    S_j^g on every nearest-neighbour bond, where g = x, y, z labels the three
    bond directions of the unit cell (Sec. 5.2 listing: the bond inside the
    cell and the two to the neighbouring cells).  Diagonal couplings per bond,
    (J + K, J, J) on x bonds and so on: an XYZ model whose couplings depend on
    the bond direction."""
    cell = UNIT_CELLS["honeycomb"]
    names = ("kx", "ky", "kz")
    inter = tuple((n,) + bond for n, bond in zip(names, cell.bonds))
    params = {n: tuple(J + (K if m == g else 0.0) for m in range(3)) for g, n in enumerate(names)}
    return Model("honeycomb-heisenberg-kitaev", cell, inter, params)


def model_kitaev_gamma(J: float = 0.0, K: float = -1.0, G: float = 0.5) -> Model:
    """Heisenberg-Kitaev-Gamma model on the honeycomb lattice (Sec. 2): on a
    bond of direction g (x, y, z as in model_heisenberg_kitaev), with (a, b)
    the other two axes, J S_i . S_j + K S_i^g S_j^g + G (S_i^a S_j^b +
    S_i^b S_j^a): a symmetric 3x3 coupling per bond direction, a general (TRI)
    model."""
    cell = UNIT_CELLS["honeycomb"]
    names = ("mx", "my", "mz")
    inter = tuple((n,) + bond for n, bond in zip(names, cell.bonds))
    params = {}
    for g, n in enumerate(names):
        a, b = (g + 1) % 3, (g + 2) % 3
        m = J * np.eye(3)
        m[g, g] += K
        m[a, b] += G
        m[b, a] += G
        params[n] = m
    return Model("honeycomb-kitaev-gamma", cell, inter, params)


def model_dm(lattice: str, J: float = 1.0, D=(0.0, 0.0, 0.3), G=None) -> Model:
    """Nearest-neighbour model on ``lattice`` with S_i . M . S_j per listed
    bond (from -> to), M = J 1 + [D]_x + G: a Dzyaloshinskii-Moriya term
    D . (S_i x S_j) (M^{ab} = eps_{abc} D_c) and an optional symmetric
    off-diagonal 3x3 part G (Sec. 2, Sec. 5.3: the bond's orientation is the
    listed one)."""
    base = model(lattice)
    m = J * np.eye(3)
    m[0, 1] += D[2]; m[1, 0] -= D[2]
    m[1, 2] += D[0]; m[2, 1] -= D[0]
    m[2, 0] += D[1]; m[0, 2] -= D[1]
    if G is not None:
        m = m + np.asarray(G, dtype=np.float64)
    params = {k: np.zeros((3, 3)) for k in base.params}
    params["j1"] = m
    return Model(f"{lattice}-dm", base.cell, base.interactions, params)


def model_compass(Jx: float = 1.0, Jy: float = 1.0) -> Model:
    """Compass model on the square lattice: Jx S^x S^x on bonds along a0 and
    Jy S^y S^y on bonds along a1 (an XYZ model with bond-dependent couplings)."""
    cell = UNIT_CELLS["square"]
    inter = (("bx",) + cell.bonds[0], ("by",) + cell.bonds[1])
    return Model("square-compass", cell, inter, {"bx": (float(Jx), 0.0, 0.0), "by": (0.0, float(Jy), 0.0)})


# ---------------------------------------------------------------- meshes ---

def log_mesh(wmin: float, wmax: float, n: int) -> np.ndarray:
    """Positive frequency mesh, logarithmically spaced (Sec. 5.1, exponential
    frequency discretization): w_n = wmin (wmax/wmin)^(n/(n-1))."""
    if n < 2:
        raise ValueError("need at least two frequencies")
    k = np.arange(n, dtype=np.float64)
    return wmin * (wmax / wmin) ** (k / (n - 1))


def exponential_schedule(lmax: float, lmin: float, b: float) -> np.ndarray:
    """Cutoff values Lambda_n = lmax b^n for n = 0 .. floor(log_b(lmin/lmax))
    (Sec. 5.1, exponential cutoff discretization)."""
    nmax = int(math.floor(math.log(lmin / lmax) / math.log(b) + 1e-12))
    return lmax * b ** np.arange(nmax + 1, dtype=np.float64)


def geometric_schedule(lmax: float, lmin: float, nsteps: int) -> np.ndarray:
    """nsteps geometric steps from lmax down to lmin inclusive."""
    k = np.arange(nsteps + 1, dtype=np.float64)
    lam = lmax * (lmin / lmax) ** (k / nsteps)
    lam[0], lam[-1] = lmax, lmin
    return lam


# -------------------------------------------------------------- workloads ---

@dataclass
class Workload:
    name: str
    lattice: str
    range: int
    params: dict
    mesh: np.ndarray
    lam_start: float
    lam_stop: float
    schedule: np.ndarray | None      # fixed-step schedule, None for adaptive
    scheme: str                      # "rk4", "dopri54" or "euler"
    kgrid: int = 0                   # k-grid side for chi(k) every step

    def model(self) -> Model:
        return model(self.lattice, **self.params)


def batch_scan_points(n: int = 64):
    """Phase-scan points: J2/J1 = k/(n-1), range 4 + (k mod 4)."""
    return [dict(j1=1.0, j2=k / (n - 1), range=4 + (k % 4)) for k in range(n)]


def _honeycomb_couplings(ndraw: int = 4):
    rng = np.random.default_rng(210913317)
    return rng.uniform(0.0, 1.0, size=(ndraw, 3))


def workload(name: str) -> Workload:
    """The five benchmark workloads (square tiny, square J1-J2, pyrochlore,
    batched square scan, honeycomb J1-J2-J3)."""
    if name == "square_tiny":
        return Workload(name, "square", 2, dict(j1=1.0), log_mesh(0.005, 50.0, 8),
                        50.0, 0.5, geometric_schedule(50.0, 0.5, 40), "rk4")
    if name == "square_j1j2":
        return Workload(name, "square", 7, dict(j1=1.0, j2=0.5), log_mesh(1e-3, 100.0, 32),
                        100.0, 0.01, None, "dopri54", kgrid=64)
    if name == "pyrochlore":
        return Workload(name, "pyrochlore", 5, dict(j1=1.0), log_mesh(1e-3, 100.0, 48),
                        100.0, 0.01, exponential_schedule(100.0, 0.01, 0.95), "rk4")
    if name == "square_scan":
        return Workload(name, "square", 7, dict(j1=1.0, j2=0.0), log_mesh(1e-3, 100.0, 24),
                        100.0, 0.01, geometric_schedule(100.0, 0.01, 120), "rk4")
    if name == "honeycomb_j123":
        j = _honeycomb_couplings()[0]
        return Workload(name, "honeycomb", 6, dict(j1=j[0], j2=j[1], j3=j[2]),
                        log_mesh(1e-3, 100.0, 32), 100.0, 0.1,
                        geometric_schedule(100.0, 0.1, 120), "rk4", kgrid=64)
    raise KeyError(name)


WORKLOAD_NAMES = ("square_tiny", "square_j1j2", "pyrochlore", "square_scan", "honeycomb_j123")


# ---------------------------------------------------------- flow states ---

def state_layout(n_freq: int, n_pairs: int) -> dict:
    """Offsets of the flow state: sigma (n_freq) | Gamma_s | Gamma_d.

    Each vertex strain is indexed [(s,u) with s >= u][t][pair]; the (s,u)
    index of mesh indices a >= c is a(a+1)/2 + c (Sec. 4.4 memory layout).
    """
    n_su = n_freq * (n_freq + 1) // 2
    per = n_su * n_freq * n_pairs
    return dict(n_su=n_su, n_triples=n_su * n_freq, vertex=per,
                sigma=0, gs=n_freq, gd=n_freq + per, size=n_freq + 2 * per)


def random_state(n_freq: int, n_pairs: int, seed: int, scale: float = 0.3, strains: int = 2) -> np.ndarray:
    """A seeded, symmetry-consistent random flow state in the layout above
    (strains = 2: sigma | Gs | Gd; strains = 4, the XYZ layout:
    sigma | Gx | Gy | Gz | Gd; strains = 16, the general layout
    sigma | G^{00} | G^{01} | ... | G^{33}).

    Im Sigma is non-positive on positive frequencies; the components whose
    second index is the density index (the last strain of the SU(2) and XYZ
    layouts, G^{mu 0} of the general one) vanish on the s = u diagonal, which
    the s<->u exchange relation forces.
    """
    lay = state_layout(n_freq, n_pairs)
    rng = np.random.default_rng(seed)
    x = np.empty(n_freq + strains * lay["vertex"], dtype=np.float64)
    x[:n_freq] = -np.abs(rng.normal(0.0, scale, n_freq))
    x[n_freq:] = rng.normal(0.0, scale, strains * lay["vertex"])
    odd = [strains - 1] if strains in (2, 4) else [q for q in range(strains) if q % 4 == 0]
    for q in odd:
        gd = x[n_freq + q * lay["vertex"]:n_freq + (q + 1) * lay["vertex"]].reshape(lay["n_su"], n_freq, n_pairs)
        for a in range(n_freq):
            gd[a * (a + 1) // 2 + a] = 0.0
    return x
