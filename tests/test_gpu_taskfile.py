"""A task file (the XML layout of Sec. 5) run end to end on the GPU: the
measured correlations equal those of a direct flow with the same mesh,
cutoffs and Euler steps bitwise, the task's calculation node records a
finished run, the lattice description file lists the lattice, and lowering the task's minimum cutoff afterwards extends the
calculation from its checkpoint (the extension of Sec. 5.1), again bitwise
equal to the direct flow, with the earlier measurements kept."""

import numpy as np
import pytest

import workloads as W
from tests.test_taskfile import RESOURCES

pytestmark = pytest.mark.gpu

TASK = """<task>
  <parameters>
    <frequency discretization="exponential"><min>0.01</min><max>40</max><count>8</count></frequency>
    <cutoff discretization="exponential"><min>{lmin}</min><max>20</max><step>0.85</step></cutoff>
    <lattice name="sq" range="2"/>
    <model name="sq-first-second" symmetry="SU2"><ja>1.0</ja><jb>0.3</jb></model>
  </parameters>
  <measurements><measurement name="correlation"/></measurements>
</task>"""


def test_task_file_runs_and_extends(tmp_path):
    import xml.etree.ElementTree as ET
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd import taskfile as T
    from paper_2109_13317_amd.flow import Context
    (tmp_path / "res.xml").write_text(RESOURCES)
    task_path = tmp_path / "run.xml"
    task_path.write_text(TASK.format(lmin=2.0))
    out = T.run(T.load(str(task_path)), scheme="euler")
    obs = str(tmp_path / "run.obs")
    first = np.load(obs)
    calc = ET.parse(str(task_path)).getroot().find("calculation").attrib
    assert calc["status"] == "finished" and "startTime" in calc and "endTime" in calc
    pos, par, bonds, inter = T.read_ldf(str(tmp_path / "run.ldf"))
    tables = build_tables(W.model("square", j1=1.0, j2=0.3), 2)
    assert len(pos) == tables.n_sites_total and int(par.sum()) == tables.n_pairs
    assert len(bonds) == 16 and len(inter) == 16 + 16    # J1 and J2 pairs within two bonds of the reference

    def direct(lmin):
        mesh = W.log_mesh(0.01, 40.0, 8)
        sched = W.exponential_schedule(20.0, lmin, 0.85)
        ctx = Context(build_tables(W.model("square", j1=1.0, j2=0.3), 2), mesh)
        x = ctx.init_state()
        ctx.flow(x, scheme="euler", schedule=sched)
        return sched, ctx.chi(sched[-1], x).cpu().numpy()

    sched, chi = direct(2.0)
    assert out[obs] == len(sched) - 1
    assert np.array_equal(first["lambda"], sched[1:])
    assert np.array_equal(first["chi_zz"][-1], chi[0]) and np.array_equal(first["chi_00"][-1], chi[1])
    # the observable-file layout: per basis site and site within range, with its metadata
    lay = first["chi_zz_sites"]
    assert lay.shape == (len(sched) - 1, tables.n_basis, tables.n_sites_total)
    np.testing.assert_array_equal(lay, T.sites_layout(tables, first["chi_zz"]))
    np.testing.assert_array_equal(first["chi_00_sites"], T.sites_layout(tables, first["chi_00"]))
    np.testing.assert_array_equal(first["sites"], tables.site_pos)
    np.testing.assert_array_equal(first["basis"], tables.basis_pos)
    assert first["lattice_vectors"].shape == (3, 3)
    # lower the minimum cutoff and run the task again: it continues from the checkpoint
    task_path.write_text(task_path.read_text().replace("<min>2.0</min>", "<min>0.5</min>"))
    T.run(T.load(str(task_path)), scheme="euler")
    second = np.load(obs)
    sched2, chi2 = direct(0.5)
    assert np.array_equal(second["lambda"], sched2[1:])
    assert np.array_equal(second["chi_zz"][:len(sched) - 1], first["chi_zz"])
    assert np.array_equal(second["chi_zz"][-1], chi2[0]) and np.array_equal(second["chi_00"][-1], chi2[1])
    assert ET.parse(str(task_path)).getroot().find("calculation").get("status") == "finished"


def test_deferred_measurement_is_computed_on_the_rerun(tmp_path):
    """method="defer" (Sec. 5.1): the flow writes the vertex state of every
    cutoff in the measurement's window instead of the measurement; running
    the finished task again computes it from them, bitwise equal to the
    same task measured directly."""
    import os
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd import taskfile as T
    from paper_2109_13317_amd.flow import Context
    (tmp_path / "res.xml").write_text(RESOURCES)
    direct = tmp_path / "direct.xml"
    direct.write_text(TASK.format(lmin=2.0).replace('<measurement name="correlation"/>',
                                                   '<measurement name="correlation" minCutoff="4"/>'))
    T.run(T.load(str(direct)), scheme="rk4")
    ref = np.load(str(tmp_path / "direct.obs"))
    deferred = tmp_path / "later.xml"
    deferred.write_text(direct.read_text().replace('minCutoff="4"', 'minCutoff="4" method="defer"'))
    out = T.run(T.load(str(deferred)), scheme="rk4")
    data = str(tmp_path / "later.data")
    assert not os.path.exists(str(tmp_path / "later.obs"))
    states = T.read_data(data)
    assert out == {data: len(ref["lambda"])} and [s[0] for s in states] == ref["lambda"].tolist()
    # the stored state of the window's last cutoff is the direct flow's there
    sched = W.exponential_schedule(20.0, 2.0, 0.85)
    k = states[-1][1]
    assert sched[k] == states[-1][0] and sched[k] >= 4.0 > sched[k + 1]
    ctx = Context(build_tables(W.model("square", j1=1.0, j2=0.3), 2), W.log_mesh(0.01, 40.0, 8))
    x = ctx.init_state()
    ctx.flow(x, scheme="rk4", schedule=sched[:k + 1])
    assert np.array_equal(states[-1][2], x.cpu().numpy())
    out = T.run(T.load(str(deferred)), scheme="rk4")
    got = np.load(str(tmp_path / "later.obs"))
    assert out[str(tmp_path / "later.obs")] == len(ref["lambda"])
    for k in ("lambda", "chi_zz", "chi_00"):
        assert np.array_equal(got[k], ref[k]), k
