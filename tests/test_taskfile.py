"""Task and resource files (the XML layout of Sec. 5) on the host: the
loader's meshes follow the paper's formulas, its unit cells and models give
the lattice front end exactly the tables the built-in models give, and
everything this SU(2) engine cannot run is refused with a clear error.  The
fixture files are written here (own model names and values)."""

import math

import numpy as np
import pytest

import workloads as W
from paper_2109_13317_amd import build_tables
from paper_2109_13317_amd import taskfile as T

RESOURCES = """
<unitcell name="sq">
  <primitive x="1" y="0" z="0"/>
  <primitive x="0" y="1" z="0"/>
  <primitive x="0" y="0" z="1"/>
  <site x="0" y="0" z="0"/>
  <bond from="0" to="0" da0="1" da1="0" da2="0"/>
  <bond from="0" to="0" da0="0" da1="1" da2="0"/>
</unitcell>
<unitcell name="hc">
  <primitive x="1.5" y="sqrt(3)/2" z="0"/>
  <primitive x="3/2" y="-sqrt(3) / 2" z="0"/>
  <primitive x="0" y="0" z="1"/>
  <site x="0" y="0" z="0"/>
  <site x="1" y="0" z="0"/>
  <bond from="0" to="1" da0="0" da1="0" da2="0"/>
  <bond from="1" to="0" da0="1" da1="0" da2="0"/>
  <bond from="1" to="0" da0="0" da1="1" da2="0"/>
</unitcell>
<model name="sq-first-second">
  <interaction parameter="ja" from="0,0,0,0" to="1,0,0,0" type="heisenberg"/>
  <interaction parameter="ja" from="0,-1,0,0" to="0,0,0,0" type="heisenberg"/>
  <interaction parameter="jb" from="0,0,0,0" to="1,1,0,0" type="heisenberg"/>
  <interaction parameter="jb" from="0,0,0,0" to="1,-1,0,0" type="heisenberg"/>
</model>
<model name="hc-first">
  <interaction parameter="j" from="0,0,0,0" to="0,0,0,1" type="heisenberg"/>
  <interaction parameter="j" from="0,0,0,1" to="1,0,0,0" type="heisenberg"/>
  <interaction parameter="j" from="0,0,0,1" to="0,1,0,0" type="heisenberg"/>
</model>
<model name="hc-anisotropic">
  <interaction parameter="j" from="0,0,0,0" to="0,0,0,1" type="xx"/>
</model>
<model name="hc-kitaev">
  <interaction parameter="j" from="0,0,0,0" to="0,0,0,1" type="heisenberg"/>
  <interaction parameter="j" from="0,0,0,0" to="0,-1,0,1" type="heisenberg"/>
  <interaction parameter="j" from="0,0,0,0" to="-1,0,0,1" type="heisenberg"/>
  <interaction parameter="k" from="0,0,0,0" to="0,0,0,1" type="xx"/>
  <interaction parameter="k" from="0,0,0,0" to="0,-1,0,1" type="yy"/>
  <interaction parameter="k" from="0,0,0,0" to="-1,0,0,1" type="zz"/>
</model>
<model name="hc-gamma">
  <interaction parameter="j" from="0,0,0,0" to="0,0,0,1" type="gx"/>
</model>
<model name="hc-kitaev-gamma">
  <interaction parameter="j" from="0,0,0,0" to="0,0,0,1" type="heisenberg"/>
  <interaction parameter="j" from="0,0,0,0" to="0,-1,0,1" type="heisenberg"/>
  <interaction parameter="j" from="0,0,0,0" to="-1,0,0,1" type="heisenberg"/>
  <interaction parameter="k" from="0,0,0,0" to="0,0,0,1" type="xx"/>
  <interaction parameter="k" from="0,0,0,0" to="0,-1,0,1" type="yy"/>
  <interaction parameter="k" from="0,0,0,0" to="-1,0,0,1" type="zz"/>
  <interaction parameter="g" from="0,0,0,0" to="0,0,0,1" type="gx"/>
  <interaction parameter="g" from="0,0,0,0" to="0,-1,0,1" type="gy"/>
  <interaction parameter="g" from="0,0,0,0" to="-1,0,0,1" type="gz"/>
</model>
<model name="sq-dm">
  <interaction parameter="j" from="0,0,0,0" to="1,0,0,0" type="heisenberg"/>
  <interaction parameter="j" from="0,0,0,0" to="0,1,0,0" type="heisenberg"/>
  <interaction parameter="d" from="0,0,0,0" to="1,0,0,0" type="xy"/>
  <interaction parameter="d" from="0,0,0,0" to="1,0,0,0" type="-yx"/>
  <interaction parameter="d" from="0,0,0,0" to="0,1,0,0" type="xy"/>
  <interaction parameter="d" from="0,0,0,0" to="0,1,0,0" type="-yx"/>
</model>
"""


def _task(tmp_path, body, name="t.xml"):
    (tmp_path / "res.xml").write_text(RESOURCES)
    p = tmp_path / name
    p.write_text(body)
    return str(p)


def _sq_task(tmp_path, ja="1.0", jb="0.4", symmetry="SU2", extra=""):
    return _task(tmp_path, f"""<task>
  <parameters>
    <frequency discretization="exponential"><min>0.01</min><max>40</max><count>9</count></frequency>
    <cutoff discretization="exponential"><min>0.5</min><max>20</max><step>0.85</step></cutoff>
    <lattice name="sq" range="3"/>
    <model name="sq-first-second" symmetry="{symmetry}"><ja>{ja}</ja><jb>{jb}</jb></model>
  </parameters>
  <measurements><measurement name="correlation" minCutoff="1.0"/></measurements>{extra}
</task>""")


def _same_tables(a, b):
    assert a.n_pairs == b.n_pairs
    for k in ("swap", "mult", "rpa_off", "rpa_ka", "rpa_kb", "rpa_cnt", "coupling", "site_pair", "site_pos",
              "basis_pos"):
        assert np.array_equal(np.asarray(getattr(a, k)), np.asarray(getattr(b, k))), k


def test_meshes_follow_the_paper_formulas(tmp_path):
    t = T.load(_sq_task(tmp_path))
    assert np.array_equal(t.mesh, W.log_mesh(0.01, 40.0, 9))
    assert np.array_equal(t.cutoffs, W.exponential_schedule(20.0, 0.5, 0.85))
    n = int(math.floor(math.log(0.5 / 20.0) / math.log(0.85)))
    assert len(t.cutoffs) == n + 1 and t.cutoffs[-1] >= 0.5
    assert t.measurements[0].min_cutoff == 1.0 and t.measurements[0].max_cutoff == math.inf
    assert t.measurements[0].method is None
    p = _task(tmp_path, """<task><parameters>
      <frequency discretization="manual"><value>0.1</value><value>1/2</value><value>3</value></frequency>
      <cutoff discretization="manual"><value>9</value><value>4</value><value>2.5</value></cutoff>
      <lattice name="hc" range="2"/><model name="hc-first" symmetry="SU2"><j>1</j></model>
    </parameters></task>""", "m.xml")
    t = T.load(p)
    assert np.array_equal(t.mesh, [0.1, 0.5, 3.0]) and np.array_equal(t.cutoffs, [9.0, 4.0, 2.5])


def test_square_model_gives_the_builtin_tables(tmp_path):
    t = T.load(_sq_task(tmp_path, ja="1.0", jb="0.4"))
    assert t.model.cell.bonds == W.unit_cell("square").bonds
    for L in (2, 3, 4):
        _same_tables(build_tables(t.model, L), build_tables(W.model("square", j1=1.0, j2=0.4), L))


def test_honeycomb_cell_with_expressions_gives_the_builtin_tables(tmp_path):
    p = _task(tmp_path, """<task><parameters>
      <frequency discretization="exponential"><min>0.01</min><max>40</max><count>4</count></frequency>
      <cutoff discretization="exponential"><min>1</min><max>10</max><step>0.5</step></cutoff>
      <lattice name="hc" range="3"/><model name="hc-first" symmetry="SU2"><j>0.7</j></model>
    </parameters></task>""")
    t = T.load(p)
    assert np.allclose(t.model.cell.primitives, W.unit_cell("honeycomb").primitives, atol=0, rtol=1e-15)
    for L in (2, 3):
        _same_tables(build_tables(t.model, L), build_tables(W.model("honeycomb", j1=0.7), L))


def test_expressions_are_arithmetic_only():
    assert T.evaluate("-sqrt(3)/2") == -math.sqrt(3.0) / 2
    assert T.evaluate("(1 + 2) * 2 ** 2") == 12.0
    assert T.evaluate("pi/4") == math.pi / 4
    for bad in ("__import__('os')", "x", "open('f')", "sqrt(1, 2)", "1 if 1 else 2", "[1]", ""):
        with pytest.raises(T.TaskError):
            T.evaluate(bad)


def test_what_the_su2_engine_cannot_run_is_refused(tmp_path):
    good = _read(_sq_task(tmp_path))
    cases = [
        (good.replace('symmetry="SU2"', 'symmetry="SU3"'), "backend"),
        (good.replace("<jb>0.4</jb>", ""), "no value"),
        (good.replace('<lattice name="sq"', '<lattice name="nowhere"'), "unitcell"),
        (good.replace("<step>0.85</step>", "<step>1.5</step>"), "step"),
        (good.replace('minCutoff="1.0"', 'method="later"'), "method"),
        (good.replace('name="correlation"', 'name="structure"'), "measurement"),
        (good.replace("<count>9</count>", "<count>1</count>"), "count"),
        (good.replace('discretization="exponential"><min>0.5', 'discretization="linear"><min>0.5'), "discretization"),
    ]
    for i, (text, msg) in enumerate(cases):
        with pytest.raises(T.TaskError, match=msg):
            T.load(_task(tmp_path, text, f"bad{i}.xml"))
    p = _task(tmp_path, """<task><parameters>
      <frequency discretization="exponential"><min>0.1</min><max>10</max><count>4</count></frequency>
      <cutoff discretization="exponential"><min>1</min><max>10</max><step>0.5</step></cutoff>
      <lattice name="hc" range="2"/><model name="hc-anisotropic" symmetry="SU2"><j>1</j></model>
    </parameters></task>""", "aniso.xml")
    with pytest.raises(T.TaskError, match="type 'xx'"):
        T.load(p)
    p = _task(tmp_path, _read(p).replace('hc-anisotropic" symmetry="SU2"', 'hc-gamma" symmetry="XYZ"'), "gamma.xml")
    with pytest.raises(T.TaskError, match="TRI"):
        T.load(p)
    (tmp_path / "dup.xml").write_text('<unitcell name="sq"><primitive x="1"/></unitcell>')
    with pytest.raises(T.TaskError, match="more than once"):
        T.load(str(tmp_path / "t.xml"))


def _read(p):
    with open(p) as f:
        return f.read()


def test_calculation_node_is_read(tmp_path):
    p = _sq_task(tmp_path, extra='\n  <calculation startTime="2026-Jan-02 03:04:05" status="running"/>')
    t = T.load(p)
    assert t.calculation == {"startTime": "2026-Jan-02 03:04:05", "status": "running"}


@pytest.mark.parametrize("lat,L,params", [
    ("square", 3, dict(j1=1.0, j2=0.4)),
    ("honeycomb", 3, dict(j1=1.0, j2=0.3, j3=-0.2)),
    ("cubic", 2, dict(j1=1.0, j2=0.5)),
    ("pyrochlore", 2, dict(j1=1.0)),
])
def test_lattice_description_by_brute_force(tmp_path, lat, L, params):
    """The lattice description (Sec. 5, "Output data") against what the
    positions alone fix: the sites are those within bond distance L of the
    reference site (bond-graph distances recomputed here from the listed
    bonds), every unordered nearest-neighbour pair of listed sites is one bond,
    every pair at a coupling shell's distance is one interaction with that
    shell's value, the parametrized sites are one per reduced pair and their
    orbits (pairs of equal distance to the reference) account for every site;
    the file reads back exactly."""
    from paper_2109_13317_amd.lattice import describe
    m = W.model(lat, **params)
    d = describe(m, L)
    t = build_tables(m, L)
    pos = d.positions
    n = len(pos)
    assert n == t.n_sites_total and np.array_equal(pos[0], t.basis_pos[0])
    dist = np.linalg.norm(pos[:, None, :] - pos[None, :, :], axis=-1)
    shells = dict(W._SHELLS[lat])
    nn = shells["j1"]
    want_bonds = {(i, j) for i in range(n) for j in range(i + 1, n) if abs(dist[i, j] - nn) < 1e-9}
    got_bonds = {tuple(sorted(b)) for b in d.bonds}
    assert len(got_bonds) == len(d.bonds) and got_bonds == want_bonds
    want_int = {}
    for name, r in W._SHELLS[lat]:
        if params.get(name, 0.0) != 0.0:
            for i in range(n):
                for j in range(i + 1, n):
                    if abs(dist[i, j] - r) < 1e-9:
                        want_int[(i, j)] = params[name]
    got_int = {tuple(sorted((i, j))): v for i, j, v in d.interactions}
    assert len(got_int) == len(d.interactions) and got_int == want_int
    # bond-graph distance from the reference site <= L for every listed site
    adj = [[] for _ in range(n)]
    for i, j in d.bonds:
        adj[i].append(j); adj[j].append(i)
    hop = {0: 0}
    frontier = [0]
    while frontier:
        nxt = []
        for i in frontier:
            for j in adj[i]:
                if j not in hop:
                    hop[j] = hop[i] + 1
                    nxt.append(j)
        frontier = nxt
    assert len(hop) == n and max(hop.values()) == L
    assert int(d.parametrized.sum()) == t.n_pairs and d.parametrized[0]
    assert int(np.sum(t.mult)) == n
    par_d = dist[0, d.parametrized]
    for r in np.unique(np.round(dist[0], 9)):          # every distance shell holds a parametrized site
        assert np.any(np.abs(par_d - r) < 1e-8)
    p = str(tmp_path / "lat.ldf")
    T.write_ldf(p, d)
    pos2, par2, bonds2, int2 = T.read_ldf(p)
    assert np.array_equal(pos2, pos) and np.array_equal(par2, d.parametrized) and bonds2 == d.bonds
    assert [(i, j) for i, j, _ in int2] == [(i, j) for i, j, _ in d.interactions]
    for (_, _, mtx), (_, _, v) in zip(int2, d.interactions):
        assert np.array_equal(mtx, np.eye(3) * v)


def test_lattice_description_layout(tmp_path):
    """Node and attribute names of the paper's lattice description layout."""
    import xml.etree.ElementTree as ET
    from paper_2109_13317_amd.lattice import describe
    p = str(tmp_path / "sq.ldf")
    T.write_ldf(p, describe(W.model("square", j1=1.0, j2=0.0), 1))
    root = ET.parse(p).getroot()
    assert root.tag == "lattice"
    assert {e.tag for e in root} == {"site", "bond", "interaction"}
    s = root.find("site")
    assert set(s.attrib) == {"id", "x", "y", "z", "parametrized"} and s.get("parametrized") == "true"
    assert len(root.findall("site")) == 5 and len(root.findall("bond")) == 4
    inter = root.findall("interaction")
    assert len(inter) == 4 and set(inter[0].attrib) == {"from", "to", "value"}
    assert inter[0].get("value") == "[[1.0,0.0,0.0], [0.0,1.0,0.0], [0.0,0.0,1.0]]"


@pytest.mark.parametrize("lat,L,params", [
    ("honeycomb", 3, dict(j1=1.0, j2=0.4, j3=0.2)),
    ("pyrochlore", 2, dict(j1=1.0)),
])
def test_observable_layout_against_the_oracle(oracle_lib, lat, L, params):
    """The per-site layout of the observable files, built from correlations
    per reduced pair, equals the oracle's correlations of every (basis site,
    site within range) of a symmetric flow, sites matched by position: the
    symmetry reduction, the site map and the site positions of the front
    end agree with the oracle's unreduced lattice."""
    import oracle
    model = W.model(lat, **params)
    tables = build_tables(model, L)
    mesh = W.log_mesh(0.05, 20.0, 4)
    orc = oracle.Oracle(model, L, mesh)
    lam = 1.5
    x = orc.flow(W.geometric_schedule(20.0, lam, 6), scheme="rk4")
    ref = orc.chi_comps(lam, x)                             # [2, nb, ns] unreduced
    # one value per reduced pair, from the first oracle site mapped to it
    pos_pair = {}
    for b in range(tables.n_basis):
        for k in range(tables.n_sites_total):
            if tables.site_pair[b, k] >= 0:
                pos_pair[(b, tuple(np.round(tables.site_pos[b, k], 6)))] = int(tables.site_pair[b, k])
    red = np.full((2, tables.n_pairs), np.nan)
    for b in range(orc.lat.nb):
        for k in range(orc.lat.nsites[b]):
            p = pos_pair[(b, tuple(np.round(orc.lat.site_pos[b, k], 6)))]
            if np.isnan(red[0, p]):
                red[:, p] = ref[:, b, k]
    assert not np.isnan(red).any()
    lay = T.sites_layout(tables, red)
    assert lay.shape == (2, tables.n_basis, tables.n_sites_total)
    scale = np.abs(ref).max()
    n = 0
    for b in range(orc.lat.nb):
        where = {tuple(np.round(orc.lat.site_pos[b, k], 6)): k for k in range(orc.lat.nsites[b])}
        for k in range(tables.n_sites_total):
            if tables.site_pair[b, k] < 0:
                assert np.isnan(lay[:, b, k]).all()
                continue
            ko = where[tuple(np.round(tables.site_pos[b, k], 6))]
            assert np.abs(lay[:, b, k] - ref[:, b, ko]).max() <= 1e-12 * scale
            n += 1
    assert n == sum(int(v) for v in orc.lat.nsites)


def _kitaev_task(tmp_path, j="0.6", k="-1.4", L=3):
    return _task(tmp_path, f"""<task><parameters>
      <frequency discretization="exponential"><min>0.01</min><max>20</max><count>6</count></frequency>
      <cutoff discretization="exponential"><min>2.0</min><max>20</max><step>0.85</step></cutoff>
      <lattice name="hc" range="{L}"/><model name="hc-kitaev" symmetry="XYZ"><j>{j}</j><k>{k}</k></model>
    </parameters>
    <measurements><measurement name="correlation"/></measurements></task>""", "kitaev.xml")


def test_xyz_task_heisenberg_kitaev_tables(tmp_path):
    """The Heisenberg-Kitaev model written as in the paper's model listing
    (Heisenberg on the three honeycomb bonds plus xx, yy, zz on one bond
    direction each) loads on the XYZ backend and gives the lattice front end
    exactly the tables of the same couplings written as one (Jx, Jy, Jz) per
    bond."""
    task = T.load(_kitaev_task(tmp_path))
    assert task.symmetry == "XYZ"
    J, K = 0.6, -1.4
    direct = W.Model("hk", W.unit_cell("honeycomb"),
                     (("x", 0, 1, 0, 0, 0), ("y", 0, 1, 0, -1, 0), ("z", 0, 1, -1, 0, 0)),
                     {"x": (J + K, J, J), "y": (J, J + K, J), "z": (J, J, J + K)})
    for L in (2, 3):
        a, b = build_tables(task.model, L), build_tables(direct, L)
        assert a.n_pairs == b.n_pairs and a.coupling.shape == (a.n_pairs, 3)
        for f in ("swap", "mult", "rpa_off", "rpa_ka", "rpa_kb", "rpa_cnt", "site_pair", "coupling", "site_pos"):
            assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_xyz_lattice_description(tmp_path):
    """The lattice description of an XYZ task lists each nonzero coupling as
    the diagonal matrix diag(Jx, Jy, Jz): the bond's x, y or z term plus the
    Heisenberg part, checked against the positions by brute force."""
    from paper_2109_13317_amd.lattice import describe
    task = T.load(_kitaev_task(tmp_path, L=2))
    path = str(tmp_path / "k.ldf")
    T.write_ldf(path, describe(task.model, 2))
    pos, par, bonds, inter = T.read_ldf(path)
    J, K = 0.6, -1.4
    cell = W.unit_cell("honeycomb")
    # bond direction of a nearest-neighbour pair from its displacement (site 0 -> site 1)
    dirs = {}
    for g, d in enumerate(((0, 0, 0), (0, -1, 0), (-1, 0, 0))):
        dirs[tuple(np.round(cell.position(d, 1) - cell.position((0, 0, 0), 0), 6))] = g
    assert len(inter) == len(bonds) > 0
    for i, j, m in inter:
        dr = tuple(np.round(pos[j] - pos[i], 6))
        g = dirs.get(dr, dirs.get(tuple(-np.asarray(dr))))
        assert g is not None
        expect = np.diag([J + (K if c == g else 0.0) for c in range(3)])
        assert np.array_equal(m, expect)


def _kitaev_gamma_task(tmp_path, j="0.2", k="-1", g="0.5", L=2, count=5):
    return _task(tmp_path, f"""<task><parameters>
      <frequency discretization="exponential"><min>0.01</min><max>20</max><count>{count}</count></frequency>
      <cutoff discretization="exponential"><min>2.0</min><max>20</max><step>0.85</step></cutoff>
      <lattice name="hc" range="{L}"/><model name="hc-kitaev-gamma" symmetry="TRI"><j>{j}</j><k>{k}</k><g>{g}</g></model>
    </parameters>
    <measurements><measurement name="correlation"/></measurements></task>""", "kitaev_gamma.xml")


def test_interaction_type_matrices():
    """The 3x3 matrices of Sec. 5.3's interaction types."""
    assert np.array_equal(T._type_matrix("heisenberg"), np.eye(3))
    assert np.array_equal(T._type_matrix("xxyy"), np.diag([1.0, 1.0, 0.0]))
    assert np.array_equal(T._type_matrix("gx"), np.array([[0, 0, 0], [0, 0, 1], [0, 1, 0.0]]))
    assert np.array_equal(T._type_matrix("gy"), np.array([[0, 0, 1], [0, 0, 0], [1, 0, 0.0]]))
    assert np.array_equal(T._type_matrix("gz"), np.array([[0, 1, 0], [1, 0, 0], [0, 0, 0.0]]))
    m = np.zeros((3, 3)); m[0, 2] = 1.0
    assert np.array_equal(T._type_matrix("xz"), m)
    assert np.array_equal(T._type_matrix("-xz"), -m)
    assert T._type_matrix("gw") is None and T._type_matrix("xw") is None


def test_tri_task_kitaev_gamma_tables(tmp_path):
    """The Kitaev-Gamma model written with heisenberg, xx/yy/zz and gx/gy/gz
    interactions loads on the TRI backend and gives the lattice front end the
    tables of the same couplings written as one matrix per bond, with and
    without spin permutations (3 pairs with them at range 2)."""
    task = T.load(_kitaev_gamma_task(tmp_path))
    assert task.symmetry == "TRI"
    J, K, G = 0.2, -1.0, 0.5
    mats = {}
    for g, name in enumerate("xyz"):
        a, b = [c for c in range(3) if c != g]
        m = J * np.eye(3)
        m[g, g] += K
        m[a, b] += G
        m[b, a] += G
        mats[name] = m
    direct = W.Model("hkg", W.unit_cell("honeycomb"),
                     (("x", 0, 1, 0, 0, 0), ("y", 0, 1, 0, -1, 0), ("z", 0, 1, -1, 0, 0)), mats)
    for sp in (False, True):
        a, b = build_tables(task.model, 2, spin_permutations=sp), build_tables(direct, 2, spin_permutations=sp)
        assert a.n_pairs == b.n_pairs and a.coupling.shape == (a.n_pairs, 3, 3)
        for f in ("swap", "mult", "rpa_off", "rpa_ka", "rpa_kb", "rpa_cnt", "site_pair", "site_pos"):
            assert np.array_equal(getattr(a, f), getattr(b, f)), f
        assert np.allclose(a.coupling, b.coupling, rtol=0, atol=1e-15)
    assert build_tables(task.model, 2, spin_permutations=True).n_pairs == 3


def test_tri_task_dm_model_and_lattice_description(tmp_path):
    """A square-lattice model with a Dzyaloshinskii-Moriya term written as xy
    and -yx interactions (Sec. 5.3): the couplings in the lattice description
    are J 1 + D (e_x e_y^T - e_y e_x^T) in the orientation the model lists
    (and its transpose backwards)."""
    from paper_2109_13317_amd.lattice import describe
    p = _task(tmp_path, """<task><parameters>
      <frequency discretization="exponential"><min>0.1</min><max>10</max><count>4</count></frequency>
      <cutoff discretization="exponential"><min>1.0</min><max>10</max><step>0.8</step></cutoff>
      <lattice name="sq" range="2"/><model name="sq-dm" symmetry="TRI"><j>1.0</j><d>0.3</d></model>
    </parameters></task>""", "dm.xml")
    task = T.load(p)
    path = str(tmp_path / "dm.ldf")
    T.write_ldf(path, describe(task.model, 2))
    pos, par, bonds, inter = T.read_ldf(path)
    want = np.eye(3) + 0.3 * np.array([[0, 1, 0], [-1, 0, 0], [0, 0, 0.0]])
    assert len(inter) == len(bonds) > 0
    for i, j, m in inter:
        dr = pos[j] - pos[i]
        assert np.isclose(abs(dr[0]) + abs(dr[1]), 1.0)
        assert np.array_equal(m, want if (dr[0] > 0.5 or dr[1] > 0.5) else want.T)

