"""Task files and resource files in the XML layout of Sec. 5 of
arXiv:2109.13317, for the SU(2) engine of this package.

A task file names the frequency mesh and the cutoff values (Sec. 5.1,
"exponential" or "manual"), a lattice (the name of a unit cell and the
truncation range), a spin model (the name of a model definition, its
numerical backend in the ``symmetry`` attribute and the values of its
coupling parameters) and the measurements.  Unit cells (Sec. 5.2:
primitive vectors, basis sites, bonds) and models (Sec. 5.3: interactions
between two sites given as four integers a0,a1,a2,b, with a coupling
parameter and a type) live in resource files: every ``*.xml`` file of a
search path is scanned for the named definitions.

What this engine accepts: the ``SU2`` backend with Heisenberg interactions
(``type="heisenberg"``), the ``XYZ`` backend with every interaction type of
diagonal matrix M (heisenberg, xxyy, xx, yy, zz, -xx, -yy, -zz: the
Heisenberg-Kitaev model of the paper's listing, for one), the ``TRI``
backend with every interaction type of Sec. 5.3 (heisenberg, xxyy, gx, gy,
gz, mu nu and -mu nu; its lattice tables use the joint lattice and spin
transformations of Sec. 4.1, as the paper's program does), and the
``correlation`` measurement (direct, or deferred to a re-run from stored
vertex states), written as a NumPy ``.npz`` file (each correlation strain
per reduced pair and cutoff, and per basis site and site within range with
the basis, lattice vectors and site positions, the data and metadata of the
paper's observable files) where the paper writes HDF5.  Anything else raises ``TaskError``.  ``run``
integrates the cutoff list (the paper's Euler steps, Eq. 42, or RK4 through
the same cutoffs) with checkpoints next to the task file and records the
calculation status (start, checkpoint and end times; running or finished)
in the task file's ``calculation`` node, as the paper's program does.  It
also writes the lattice description file (task path with extension
``.ldf``): the sites within range of the reference site, which of them are
parametrized, the bonds and the interactions (``write_ldf``).
"""

from __future__ import annotations

import ast
import datetime
import glob
import math
import operator
import os
import xml.etree.ElementTree as ET
from dataclasses import dataclass, field

import numpy as np


class TaskError(ValueError):
    """A task or resource file this engine cannot run."""


# ------------------------------------------------------------ expressions --

_OPS = {ast.Add: operator.add, ast.Sub: operator.sub, ast.Mult: operator.mul, ast.Div: operator.truediv,
        ast.Pow: operator.pow, ast.USub: operator.neg, ast.UAdd: operator.pos}
_FUNCS = {"sqrt": math.sqrt, "sin": math.sin, "cos": math.cos, "tan": math.tan}
_CONSTS = {"pi": math.pi}


def evaluate(expr: str) -> float:
    """Value of an arithmetic coordinate expression such as ``3/2`` or
    ``-sqrt(3)/2``: numbers, + - * / **, parentheses, sqrt/sin/cos/tan and
    pi; nothing else is evaluated."""
    def ev(node):
        if isinstance(node, ast.Expression):
            return ev(node.body)
        if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
            return float(node.value)
        if isinstance(node, ast.BinOp) and type(node.op) in _OPS:
            return _OPS[type(node.op)](ev(node.left), ev(node.right))
        if isinstance(node, ast.UnaryOp) and type(node.op) in _OPS:
            return _OPS[type(node.op)](ev(node.operand))
        if isinstance(node, ast.Name) and node.id in _CONSTS:
            return _CONSTS[node.id]
        if (isinstance(node, ast.Call) and isinstance(node.func, ast.Name) and node.func.id in _FUNCS
                and len(node.args) == 1 and not node.keywords):
            return _FUNCS[node.func.id](ev(node.args[0]))
        raise TaskError(f"unsupported expression {expr!r}")
    try:
        tree = ast.parse(expr.strip(), mode="eval")
    except SyntaxError as e:
        raise TaskError(f"unsupported expression {expr!r}") from e
    return float(ev(tree))


# ------------------------------------------------------------ definitions --

@dataclass(frozen=True)
class UnitCellDef:
    """A unit cell (Sec. 5.2): rows of ``primitives`` are a0, a1, a2; bonds
    are (from, to, da0, da1, da2)."""
    name: str
    primitives: np.ndarray
    basis: np.ndarray
    bonds: tuple

    @property
    def n_basis(self) -> int:
        return int(self.basis.shape[0])

    def position(self, cell, b) -> np.ndarray:
        """Cartesian position of basis site b in the cell (a0, a1, a2)."""
        return np.asarray(cell, dtype=np.float64) @ self.primitives + self.basis[b]


@dataclass(frozen=True)
class ModelDef:
    """Heisenberg couplings (Sec. 5.3) as the lattice front end takes them:
    interactions (parameter, b_from, b_to, da0, da1, da2) with the first site
    in cell 0, and the parameter values."""
    name: str
    cell: UnitCellDef
    interactions: tuple
    params: dict = field(default_factory=dict)


@dataclass
class Measurement:
    name: str
    output: str | None = None
    min_cutoff: float = 0.0
    max_cutoff: float = math.inf
    method: str | None = None


@dataclass
class Task:
    path: str
    mesh: np.ndarray            # positive frequencies, ascending
    cutoffs: np.ndarray         # cutoff values in the order of the flow
    lattice_range: int
    model: ModelDef
    symmetry: str
    measurements: list
    calculation: dict           # attributes of the calculation node ({} if none)


def _child_text(node, tag, path):
    c = node.find(tag)
    if c is None or c.text is None:
        raise TaskError(f"{path}: <{node.tag}> needs <{tag}>")
    return c.text


def _discretization(node, path, kind):
    how = node.get("discretization")
    if how == "manual":
        vals = [evaluate(v.text) for v in node.findall("value")]
        if len(vals) < 2:
            raise TaskError(f"{path}: manual <{kind}> needs at least two values")
        return np.asarray(vals, dtype=np.float64)
    if how != "exponential":
        raise TaskError(f"{path}: <{kind}> discretization must be exponential or manual")
    lo = evaluate(_child_text(node, "min", path))
    hi = evaluate(_child_text(node, "max", path))
    if not (0.0 < lo < hi):
        raise TaskError(f"{path}: <{kind}> needs 0 < min < max")
    if kind == "frequency":
        n = int(_child_text(node, "count", path))
        if n < 2:
            raise TaskError(f"{path}: <frequency> needs count >= 2")
        k = np.arange(n, dtype=np.float64)
        return lo * (hi / lo) ** (k / (n - 1))
    b = evaluate(_child_text(node, "step", path))
    if not (0.0 < b < 1.0):
        raise TaskError(f"{path}: <cutoff> step must lie in (0, 1)")
    nmax = int(math.floor(math.log(lo / hi) / math.log(b) + 1e-12))
    return hi * b ** np.arange(nmax + 1, dtype=np.float64)


def _resource_nodes(search_path, tag, name):
    found = []
    for d in search_path:
        for f in sorted(glob.glob(os.path.join(d, "*.xml"))):
            try:
                text = open(f).read()
            except OSError:
                continue
            try:
                root = ET.fromstring(f"<resources>{text}</resources>")
            except ET.ParseError as e:
                raise TaskError(f"{f}: not well-formed XML ({e})") from e
            # definitions are top-level elements (a task file's nested
            # <model> node is a reference, not a definition)
            found += [(f, n) for n in root.findall(tag) if n.get("name") == name]
    if not found:
        raise TaskError(f"no <{tag} name=\"{name}\"> in the resource files of {list(search_path)}")
    if len(found) > 1:
        raise TaskError(f"<{tag} name=\"{name}\"> is defined more than once: {[f for f, _ in found]}")
    return found[0]


def _unit_cell(search_path, name):
    f, node = _resource_nodes(search_path, "unitcell", name)
    prims = [[evaluate(p.get(c, "0")) for c in "xyz"] for p in node.findall("primitive")]
    if len(prims) != 3:
        raise TaskError(f"{f}: unit cell {name!r} needs three primitive vectors")
    basis = [[evaluate(s.get(c, "0")) for c in "xyz"] for s in node.findall("site")]
    if not basis:
        raise TaskError(f"{f}: unit cell {name!r} has no sites")
    bonds = []
    for bnd in node.findall("bond"):
        b = tuple(int(bnd.get(k, "0")) for k in ("from", "to", "da0", "da1", "da2"))
        if not (0 <= b[0] < len(basis) and 0 <= b[1] < len(basis)):
            raise TaskError(f"{f}: bond of unit cell {name!r} names a missing site")
        bonds.append(b)
    return UnitCellDef(name, np.asarray(prims, dtype=np.float64), np.asarray(basis, dtype=np.float64),
                       tuple(bonds))


# Interaction types with a diagonal matrix M (Sec. 5.3): what the XYZ backend
# takes; the off-diagonal ones (gx, gy, gz, mu nu with mu != nu) need the
# TRI backend (_type_matrix).
_DIAGONAL_TYPES = {"heisenberg": (1.0, 1.0, 1.0), "xxyy": (1.0, 1.0, 0.0),
                   "xx": (1.0, 0.0, 0.0), "yy": (0.0, 1.0, 0.0), "zz": (0.0, 0.0, 1.0),
                   "-xx": (-1.0, 0.0, 0.0), "-yy": (0.0, -1.0, 0.0), "-zz": (0.0, 0.0, -1.0)}


_AXES = {"x": 0, "y": 1, "z": 2}


def _type_matrix(kind: str):
    """The 3x3 matrix M of an interaction type (Sec. 5.3): heisenberg, xxyy,
    gx, gy, gz (the symmetric off-diagonal Gamma terms), mu nu (a single 1 at
    row mu, column nu) and -mu nu; None for an unknown type."""
    if kind == "heisenberg":
        return np.eye(3)
    if kind == "xxyy":
        return np.diag([1.0, 1.0, 0.0])
    if len(kind) == 2 and kind[0] == "g" and kind[1] in _AXES:
        a, b = [c for c in range(3) if c != _AXES[kind[1]]]
        m = np.zeros((3, 3))
        m[a, b] = m[b, a] = 1.0
        return m
    sign = 1.0
    if kind.startswith("-"):
        sign, kind = -1.0, kind[1:]
    if len(kind) == 2 and kind[0] in _AXES and kind[1] in _AXES:
        m = np.zeros((3, 3))
        m[_AXES[kind[0]], _AXES[kind[1]]] = sign
        return m
    return None


def _model(search_path, name, cell, params, symmetry="SU2"):
    """The model's interactions with the first site in cell 0.  SU2: every
    interaction is Heisenberg, parameters are numbers.  XYZ: every
    interaction has a diagonal matrix M; each (parameter, type) becomes a
    coupling (Jx, Jy, Jz) = value x diag(M).  TRI: each (parameter, type)
    becomes the coupling matrix value x M."""
    f, node = _resource_nodes(search_path, "model", name)
    inter = []
    vec = {}
    for it in node.findall("interaction"):
        kind = it.get("type", "")
        if symmetry == "SU2" and kind != "heisenberg":
            raise TaskError(f"{f}: interaction type {kind!r} needs a backend other than SU2")
        if symmetry == "XYZ" and kind not in _DIAGONAL_TYPES:
            raise TaskError(f"{f}: interaction type {kind!r} couples different spin components (TRI backend)")
        if symmetry == "TRI" and _type_matrix(kind) is None:
            raise TaskError(f"{f}: unknown interaction type {kind!r}")
        src = [int(v) for v in it.get("from", "").split(",")]
        dst = [int(v) for v in it.get("to", "").split(",")]
        if len(src) != 4 or len(dst) != 4:
            raise TaskError(f"{f}: interaction sites are a0,a1,a2,b")
        if not (0 <= src[3] < cell.n_basis and 0 <= dst[3] < cell.n_basis):
            raise TaskError(f"{f}: interaction names a missing basis site")
        p = it.get("parameter")
        if p not in params:
            raise TaskError(f"the task gives no value for the model parameter {p!r}")
        if symmetry == "XYZ":
            key = f"{p}:{kind}"
            vec[key] = tuple(float(params[p]) * m for m in _DIAGONAL_TYPES[kind])
            p = key
        elif symmetry == "TRI":
            key = f"{p}:{kind}"
            vec[key] = float(params[p]) * _type_matrix(kind)
            p = key
        inter.append((p, src[3], dst[3], dst[0] - src[0], dst[1] - src[1], dst[2] - src[2]))
    return ModelDef(name, cell, tuple(inter), vec if symmetry in ("XYZ", "TRI") else dict(params))


def load(path: str, search_path=None) -> Task:
    """Read a task file and the resource files it references (default
    search path: the task file's directory and its ``res`` subdirectory)."""
    try:
        root = ET.parse(path).getroot()
    except (OSError, ET.ParseError) as e:
        raise TaskError(f"{path}: {e}") from e
    if root.tag != "task":
        raise TaskError(f"{path}: the top-level node must be <task>")
    if search_path is None:
        here = os.path.dirname(os.path.abspath(path))
        search_path = [here, os.path.join(here, "res")]
    par = root.find("parameters")
    if par is None:
        raise TaskError(f"{path}: <task> needs <parameters>")
    nodes = {t: par.find(t) for t in ("frequency", "cutoff", "lattice", "model")}
    for t, n in nodes.items():
        if n is None:
            raise TaskError(f"{path}: <parameters> needs <{t}>")
    mesh = _discretization(nodes["frequency"], path, "frequency")
    if not (mesh > 0).all() or not (np.diff(mesh) > 0).all():
        raise TaskError(f"{path}: frequencies must be positive and ascending")
    cut = _discretization(nodes["cutoff"], path, "cutoff")
    if not (cut > 0).all() or not (np.diff(cut) < 0).all():
        raise TaskError(f"{path}: cutoff values must be positive and descending")
    lat, mod = nodes["lattice"], nodes["model"]
    symmetry = mod.get("symmetry", "")
    if symmetry not in ("SU2", "XYZ", "TRI"):
        raise TaskError(f"{path}: backend {symmetry!r} is not available (this engine runs SU2, XYZ and TRI)")
    params = {c.tag: evaluate(c.text) for c in mod if c.text is not None}
    cell = _unit_cell(search_path, lat.get("name"))
    model = _model(search_path, mod.get("name"), cell, params, symmetry)
    meas = []
    mnode = root.find("measurements")
    for m in (mnode.findall("measurement") if mnode is not None else []):
        if m.get("name") != "correlation":
            raise TaskError(f"{path}: unknown measurement {m.get('name')!r}")
        if m.get("method") not in (None, "direct", "defer"):
            raise TaskError(f"{path}: measurement method {m.get('method')!r} is not available")
        meas.append(Measurement("correlation", m.get("output"),
                                evaluate(m.get("minCutoff", "0")),
                                evaluate(m.get("maxCutoff", "inf")) if m.get("maxCutoff") else math.inf,
                                m.get("method")))
    calc = root.find("calculation")
    return Task(os.path.abspath(path), mesh, cut, int(lat.get("range", "-1")), model, symmetry, meas,
                dict(calc.attrib) if calc is not None else {})


def _stamp() -> str:
    return datetime.datetime.now().strftime("%Y-%b-%d %H:%M:%S")


def _set_calculation(path: str, **attrs) -> None:
    tree = ET.parse(path)
    root = tree.getroot()
    calc = root.find("calculation")
    if calc is None:
        calc = ET.SubElement(root, "calculation")
    for k, v in attrs.items():
        calc.set(k, v)
    tmp = path + ".tmp"
    tree.write(tmp)
    os.replace(tmp, path)


def write_ldf(path: str, desc) -> None:
    """Write a ``lattice.LatticeDescription`` as a lattice description file
    (the XML layout of Sec. 5, "Output data": a ``lattice`` root with
    ``site`` nodes (id, Cartesian x, y, z, parametrized), ``bond`` nodes
    (from, to) and ``interaction`` nodes (from, to, the 3x3 coupling matrix
    row by row); numbers are written exactly, as Python's shortest round-trip
    decimal)."""
    root = ET.Element("lattice")
    for i, (p, par) in enumerate(zip(desc.positions, desc.parametrized)):
        ET.SubElement(root, "site", id=str(i), x=repr(float(p[0])), y=repr(float(p[1])), z=repr(float(p[2])),
                      parametrized="true" if par else "false")
    for i, j in desc.bonds:
        ET.SubElement(root, "bond", **{"from": str(i), "to": str(j)})
    for i, j, v in desc.interactions:
        m = np.asarray(v) if np.ndim(v) == 2 else (np.diag(v) if np.ndim(v) == 1 else np.eye(3) * v)
        val = "[" + ", ".join("[" + ",".join(repr(float(e)) for e in row) + "]" for row in m) + "]"
        ET.SubElement(root, "interaction", value=val, **{"from": str(i), "to": str(j)})
    ET.indent(root)
    tmp = path + ".tmp"
    ET.ElementTree(root).write(tmp)
    os.replace(tmp, path)


def read_ldf(path: str):
    """Read a lattice description file back: (positions [n, 3], parametrized
    [n], bonds [(from, to)], interactions [(from, to, 3x3 matrix)])."""
    try:
        root = ET.parse(path).getroot()
    except (ET.ParseError, OSError) as e:
        raise TaskError(f"{path}: {e}") from None
    sites = sorted(root.findall("site"), key=lambda e: int(e.get("id")))
    if [int(e.get("id")) for e in sites] != list(range(len(sites))):
        raise TaskError(f"{path}: site ids are not 0..n-1")
    pos = np.array([[float(e.get(k)) for k in "xyz"] for e in sites]).reshape(-1, 3)
    par = np.array([e.get("parametrized") == "true" for e in sites], dtype=bool)
    bonds = [(int(e.get("from")), int(e.get("to"))) for e in root.findall("bond")]
    inter = []
    for e in root.findall("interaction"):
        rows = e.get("value").strip()[1:-1].replace(" ", "").split("],[")
        m = np.array([[float(v) for v in r.strip("[]").split(",")] for r in rows])
        if m.shape != (3, 3):
            raise TaskError(f"{path}: interaction value is not a 3x3 matrix")
        inter.append((int(e.get("from")), int(e.get("to")), m))
    return pos, par, bonds, inter


def _write_state(dest, lam, index, state) -> None:
    tmp = dest + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, **{"lambda": np.float64(lam), "index": np.int64(index), "state": state})
    os.replace(tmp, dest)


def read_data(path: str):
    """The vertex states a deferred measurement left in ``path`` (the task
    path with extension ``.data``): [(cutoff, schedule index, state)] in the
    order of the flow."""
    out = []
    for f in sorted(glob.glob(os.path.join(path, "*.npz"))):
        with np.load(f, allow_pickle=False) as z:
            out.append((float(z["lambda"]), int(z["index"]), np.array(z["state"], dtype=np.float64)))
    return out


def sites_layout(tables, chi_pairs) -> np.ndarray:
    """Correlations per reduced pair [..., n_pairs] spread onto the layout of
    the paper's observable files (Sec. 5, "Output data"): for every basis
    site b of the unit cell, every site k within range of it, [...,
    n_basis, n_sites_total]; slots past a basis site's own site count hold
    NaN.  With spin rotations (tables reduced by spin permutations) the
    sixteen components [..., 16, n_pairs] of each site are rotated:
    W chi W^T on the spin indices."""
    c = np.asarray(chi_pairs, dtype=np.float64)
    sp = np.asarray(tables.site_pair)
    out = np.full(c.shape[:-1] + sp.shape, np.nan)
    ok = sp >= 0
    out[..., ok] = c[..., sp[ok]]
    if getattr(tables, "rot", None) is not None:
        assert c.shape[-2] == 16, "rotated layouts need all sixteen components"
        for b, k in zip(*np.nonzero(ok)):
            R4 = np.eye(4)
            R4[1:, 1:] = tables.rot[tables.site_rot[b, k]]
            v = c[..., sp[b, k]].reshape(c.shape[:-2] + (4, 4))
            out[..., b, k] = np.einsum("ma,...ab,nb->...mn", R4, v, R4).reshape(c.shape[:-1])
    return out


def chi_names(nc: int) -> tuple:
    """Names of the correlation strains in the measurement files: SU2 chi^zz
    and chi^00, XYZ chi^xx, chi^yy, chi^zz and chi^00, TRI every chi^{mu nu}
    (chi_00, chi_0x, ..., chi_zz, in the order 4 mu + nu)."""
    if nc == 16:
        return tuple("chi_" + "0xyz"[m // 4] + "0xyz"[m % 4] for m in range(16))
    return ("chi_zz", "chi_00") if nc == 2 else ("chi_xx", "chi_yy", "chi_zz", "chi_00")


def _write_obs(dest, rec, tables=None, cell=None) -> None:
    """The correlation measurement: cutoffs and every strain per reduced
    pair (``chi_names``; rec = (cutoffs, [strains, pairs] per cutoff)), and
    (with the lattice tables) the same in the observable layout of Sec. 5
    (``<name>_sites``: [cutoff, basis site, site within range]) with its
    metadata (``basis``, ``lattice_vectors``, ``sites``: Cartesian
    positions)."""
    chis = [np.asarray(c, dtype=np.float64) for c in rec[1]]
    nc = chis[0].shape[0] if chis else ({1: 2, 2: 4, 3: 16}[np.ndim(tables.coupling)] if tables is not None else 2)
    arrays = {"lambda": np.asarray(rec[0], dtype=np.float64)}
    for m, name in enumerate(chi_names(nc)):
        arrays[name] = np.array([c[m] for c in chis]) if chis else np.zeros((0, 0))
    if tables is not None:
        nb, ns_tot = np.asarray(tables.site_pair).shape
        lay = sites_layout(tables, np.array(chis)) if chis else None      # [cutoff, strain, nb, ns_tot]
        for m, name in enumerate(chi_names(nc)):
            arrays[name + "_sites"] = lay[:, m] if chis else np.zeros((0, nb, ns_tot))
        arrays["basis"] = np.asarray(tables.basis_pos, dtype=np.float64)
        arrays["sites"] = np.asarray(tables.site_pos, dtype=np.float64)
        if cell is not None:
            arrays["lattice_vectors"] = np.asarray(cell.primitives, dtype=np.float64)
    tmp = dest + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, **arrays)
    os.replace(tmp, dest)


def run(task: Task, *, scheme: str = "euler", precision: str = "fp64", every: float = 3600.0,
        force_restart: bool = False) -> dict:
    """Integrate a loaded task along its cutoff values (``euler`` as in the
    paper, or ``rk4`` through the same cutoffs) on the GPU, with checkpoints
    in the task path with extension ``.checkpoint`` (a snapshot at least
    ``every`` seconds apart, and at the end), and write each correlation
    measurement (default output: the task path with extension ``.obs``; a
    NumPy archive with ``lambda`` and each strain per reduced pair, SU2
    ``chi_zz``, ``chi_00``, XYZ ``chi_xx``, ``chi_yy``, ``chi_zz``,
    ``chi_00``, and the same per basis site and site within range as the
    paper's observable files hold them, ``_write_obs``), updated after every
    accepted step, and the lattice description
    in the task path with extension ``.ldf`` (``write_ldf``).  A measurement
    with ``method="defer"`` (Sec. 5.1) records nothing during the flow: the
    vertex state of each of its cutoffs goes to the directory with the task
    path and extension ``.data`` (one ``.npz`` per cutoff, ``read_data``),
    and running the finished task again computes the measurement from them.
    A task with a snapshot of the
    same calculation resumes from it (measurements up to the snapshot are kept
    and the rest recomputed; the resumed steps are bitwise the uninterrupted
    ones) unless ``force_restart``.  Returns {output path: cutoffs recorded},
    with {data path: states stored in this call} for deferred measurements
    not yet computed."""
    from . import checkpoint
    from .flow import Context
    from .lattice import build_tables, describe

    if task.lattice_range < 0:
        raise TaskError(f"{task.path}: <lattice> needs a range")
    if scheme not in ("euler", "rk4"):
        raise TaskError("scheme must be euler or rk4")
    base = os.path.splitext(task.path)[0]
    ck = base + ".checkpoint"
    dests = []
    for m in task.measurements:
        d = m.output or base + ".obs"
        dests.append(d if os.path.isabs(d) else os.path.join(os.path.dirname(task.path), d))
    records = [([], []) for _ in task.measurements]
    names = chi_names({"SU2": 2, "XYZ": 4, "TRI": 16}[task.symmetry])
    resuming = os.path.exists(ck) and not force_restart
    if resuming:
        lam_snap = float.fromhex(checkpoint.read(ck).meta["lambda"])
        for rec, d in zip(records, dests):
            if os.path.exists(d):
                with np.load(d, allow_pickle=False) as z:
                    keep = z["lambda"] >= lam_snap
                    rec[0].extend(z["lambda"][keep].tolist())
                    rec[1].extend(list(np.stack([z[n][keep] for n in names], axis=1)))
    write_ldf(base + ".ldf", describe(task.model, task.lattice_range))
    tables = build_tables(task.model, task.lattice_range, spin_permutations=task.symmetry == "TRI")
    ctx = Context(tables, task.mesh, precision=precision)
    x = ctx.init_state()
    defer = [m.method == "defer" for m in task.measurements]
    data_dir = base + ".data"
    index_of = {float(v): i for i, v in enumerate(task.cutoffs)}
    stored = [0]

    def observe(lam, chi, chik):
        c = chi.detach().cpu().numpy()
        keep_state = False
        for m, rec, d, dfr in zip(task.measurements, records, dests, defer):
            if m.min_cutoff <= lam <= m.max_cutoff:
                if dfr:
                    keep_state = True
                    continue
                rec[0].append(lam)
                rec[1].append(c.copy())
                _write_obs(d, rec, tables, task.model.cell)
        if keep_state:
            os.makedirs(data_dir, exist_ok=True)
            i = index_of.get(float(lam))
            if i is None:
                i = int(np.argmin(np.abs(np.asarray(task.cutoffs) - lam)))
            _write_state(os.path.join(data_dir, f"{i:06d}.npz"), lam, i, x.detach().cpu().numpy())
            stored[0] += 1
        return False

    started = task.calculation.get("startTime") if resuming else None
    _set_calculation(task.path, startTime=started or _stamp(), status="running")
    n = checkpoint.flow(ctx, x, ck, scheme=scheme, schedule=list(task.cutoffs), every=every, observer=observe,
                        force_restart=force_restart)
    snap = checkpoint.read(ck).meta
    now = _stamp()
    finished = snap["status"] == "finished"
    _set_calculation(task.path, checkpointTime=now, endTime=now, status="finished" if finished else "running")
    out = {}
    if any(defer) and finished and n == 0:
        # a re-run of a finished calculation: the deferred measurements, from
        # the stored vertex states
        import torch
        for lam, _, state in read_data(data_dir):
            c = ctx.chi(lam, torch.from_numpy(state).cuda()).cpu().numpy()
            for m, rec, dfr in zip(task.measurements, records, defer):
                if dfr and m.min_cutoff <= lam <= m.max_cutoff:
                    rec[0].append(lam)
                    rec[1].append(c.copy())
        for rec, d, dfr in zip(records, dests, defer):
            if dfr:
                _write_obs(d, rec, tables, task.model.cell)
                out[d] = len(rec[0])
    elif stored[0]:
        out[data_dir] = stored[0]
    for rec, d, dfr in zip(records, dests, defer):
        if not dfr:
            _write_obs(d, rec, tables, task.model.cell)
            out[d] = len(rec[0])
    return out
