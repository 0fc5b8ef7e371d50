"""Checkpoint/resume and task-file runs against the FP64 oracle.

The calculation node of a task (Sec. 5.1) can stop and continue a flow, or
extend a finished one to lower cutoffs; the results must be those of the
flow equations integrated without interruption.  Here the reference is the
oracle's own uninterrupted flow, not the library's:
  * an adaptive Dormand-Prince flow stopped after 7 accepted steps and
    resumed from its snapshot with a fresh state tensor: same accepted
    cutoffs as oracle.dopri_flow, final state within 1e-10;
  * a fixed RK4 flow run on the first 20 cutoffs, then extended from its
    snapshot to the whole schedule: within 1e-10 of oracle.flow;
  * a task file (the XML layout of Sec. 5) run with Euler steps (Eq. 42):
    chi per pair at every cutoff within 1e-10 of the oracle's Euler flow.
"""

import numpy as np
import pytest

import workloads as W
from tests.parity import compare_chi, compare_vertex

pytestmark = pytest.mark.gpu

TOL = 1e-10
MESH = W.log_mesh(0.005, 50.0, 8)
MODEL = dict(j1=1.0, j2=0.5)
ADAPT = dict(scheme="dopri54", lam_start=50.0, lam_stop=0.5, rtol=1e-5, atol=1e-8, h0=0.05, hmin=1e-10)
SCHED = list(20.0 * 0.85 ** np.arange(38))        # 20 -> 0.0095


def _say(*a):
    print(*a, flush=True)


def _setup():
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    model = W.model("square", **MODEL)
    tables = build_tables(model, 2)
    return tables, Context(tables, MESH), oracle.Oracle(model, 2, MESH)


class _Record:
    def __init__(self, stop_after=0):
        self.lams, self.stop_after = [], stop_after

    def __call__(self, lam, chi, chik):
        self.lams.append(lam)
        return bool(self.stop_after) and len(self.lams) >= self.stop_after


def test_resumed_adaptive_flow_matches_oracle(tmp_path):
    from paper_2109_13317_amd import checkpoint as C
    tables, ctx, orc = _setup()
    p = str(tmp_path / "a.checkpoint")
    first = _Record(stop_after=7)
    x = ctx.init_state()
    assert C.flow(ctx, x, p, every=0.0, observer=first, **ADAPT) == 7
    assert C.read(p).meta["status"] == "running"
    rest = _Record()
    x2 = ctx.init_state()                                  # the state comes from the snapshot
    n2 = C.flow(ctx, x2, p, every=0.0, observer=rest, **ADAPT)
    xo, lams = orc.dopri_flow(ADAPT["lam_start"], ADAPT["lam_stop"], ADAPT["rtol"], ADAPT["atol"], ADAPT["h0"],
                              ADAPT["hmin"])
    got = first.lams + rest.lams
    _say(f"resumed adaptive flow: 7 + {n2} steps, oracle {len(lams)}")
    assert len(got) == len(lams) == 7 + n2
    assert np.abs(np.array(got) - np.array(lams)).max() <= 1e-12 * ADAPT["lam_start"]
    err = compare_vertex(orc, tables, xo, x2.cpu().numpy())
    _say(f"  final state vs oracle {err:.2e}")
    assert err <= TOL


def test_extended_fixed_flow_matches_oracle(tmp_path):
    from paper_2109_13317_amd import checkpoint as C
    tables, ctx, orc = _setup()
    p = str(tmp_path / "f.checkpoint")
    x = ctx.init_state()
    assert C.flow(ctx, x, p, scheme="rk4", schedule=SCHED[:20], every=0.0) == 19
    assert C.read(p).meta["status"] == "finished"
    x2 = ctx.init_state()
    assert C.flow(ctx, x2, p, scheme="rk4", schedule=SCHED, every=0.0) == len(SCHED) - 20
    xo = orc.flow(SCHED, scheme="rk4")
    err = compare_vertex(orc, tables, xo, x2.cpu().numpy())
    _say(f"extended RK4 flow ({len(SCHED) - 1} steps) vs oracle {err:.2e}")
    assert err <= TOL


def test_task_file_run_matches_oracle(tmp_path):
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd import taskfile as T
    from tests.test_gpu_taskfile import TASK
    from tests.test_taskfile import RESOURCES
    (tmp_path / "res.xml").write_text(RESOURCES)
    task_path = tmp_path / "run.xml"
    task_path.write_text(TASK.format(lmin=2.0))
    T.run(T.load(str(task_path)), scheme="euler")
    got = np.load(str(tmp_path / "run.obs"))
    # the task's lattice ('sq', range 2) and model (first and second
    # neighbours, 1.0 and 0.3) on the oracle, with the task's mesh and cutoffs
    model = W.model("square", j1=1.0, j2=0.3)
    mesh = W.log_mesh(0.01, 40.0, 8)
    sched = W.exponential_schedule(20.0, 2.0, 0.85)
    orc = oracle.Oracle(model, 2, mesh)
    tables = build_tables(model, 2)
    ref = []
    orc.flow(sched, scheme="euler", observer=lambda lam, xs: ref.append((lam, orc.chi(lam, xs))))
    assert np.array_equal(got["lambda"], sched[1:]) and len(ref) == len(sched) - 1
    worst = 0.0
    for i, (lam, (zz, dd)) in enumerate(ref):
        assert got["lambda"][i] == lam
        red = np.stack([got["chi_zz"][i], got["chi_00"][i]])
        worst = max(worst, compare_chi(orc, tables, zz, dd, red))
    _say(f"task-file run: chi at {len(ref)} cutoffs, worst error vs oracle {worst:.2e}")
    assert worst <= TOL


def test_xyz_task_file_run_matches_oracle(tmp_path):
    """A task on the XYZ backend: the Heisenberg-Kitaev model written as in
    the paper's model listing (j = 0.6, k = -1.4, honeycomb range 3), Euler
    steps; the four correlation strains at every cutoff, per reduced pair and
    in the observable-file layout, against the oracle's XYZ Euler flow."""
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd import taskfile as T
    from tests.parity import compare_chi_comps, compare_chi_sites
    from tests.test_taskfile import _kitaev_task
    path = _kitaev_task(tmp_path)
    task = T.load(path)
    T.run(task, scheme="euler")
    got = np.load(path[:-4] + ".obs")
    tables = build_tables(task.model, 3)
    orc = oracle.Oracle(task.model, 3, task.mesh)
    assert orc.nc == 4
    ref = []
    orc.flow(task.cutoffs, scheme="euler", observer=lambda lam, xs: ref.append((lam, orc.chi_comps(lam, xs))))
    assert np.array_equal(got["lambda"], task.cutoffs[1:]) and len(ref) == len(task.cutoffs) - 1
    names = T.chi_names(4)
    worst = 0.0
    for i, (lam, cc) in enumerate(ref):
        red = np.stack([got[n][i] for n in names])
        worst = max(worst, compare_chi_comps(orc, tables, cc, red))
        lay = np.stack([got[n + "_sites"][i] for n in names])
        worst = max(worst, compare_chi_sites(orc, tables, lay, cc, red))
    _say(f"XYZ task-file run ({tables.n_pairs} pairs): chi at {len(ref)} cutoffs, worst error vs oracle {worst:.2e}")
    assert worst <= TOL


def test_tri_task_file_run_matches_oracle(tmp_path):
    """A task on the TRI backend: the Kitaev-Gamma model written with
    heisenberg, xx/yy/zz and gx/gy/gz interactions (honeycomb range 2; the
    task's tables use spin permutations, 3 pairs), Euler steps; all sixteen
    correlation components at every cutoff, per reduced pair (rotated onto
    every site) and in the observable-file layout, against the oracle's
    TRI Euler flow on the unreduced lattice."""
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd import taskfile as T
    from tests.parity import compare_chi_rot
    from tests.test_taskfile import _kitaev_gamma_task
    path = _kitaev_gamma_task(tmp_path)
    task = T.load(path)
    T.run(task, scheme="euler")
    got = np.load(path[:-4] + ".obs")
    tables = build_tables(task.model, 2, spin_permutations=True)
    orc = oracle.Oracle(task.model, 2, task.mesh)
    assert orc.nc == 16 and tables.n_pairs == 3
    ref = []
    orc.flow(task.cutoffs, scheme="euler",
             observer=lambda lam, xs: ref.append((lam, orc.chi_tri(lam, xs)[0].reshape(16, orc.lat.nb, orc.lat.ns))))
    assert np.array_equal(got["lambda"], task.cutoffs[1:]) and len(ref) == len(task.cutoffs) - 1
    names = T.chi_names(16)
    worst = 0.0
    for i, (lam, cc) in enumerate(ref):
        red = np.stack([got[n][i] for n in names])
        worst = max(worst, compare_chi_rot(orc, tables, cc, red))
        lay = np.stack([got[n + "_sites"][i] for n in names])
        scale = np.abs(cc).max()
        for b in range(tables.n_basis):
            where = {tuple(np.round(orc.lat.site_pos[b, k], 6)): k for k in range(orc.lat.nsites[b])}
            for k in range(tables.n_sites_total):
                if tables.site_pair[b, k] < 0:
                    assert np.isnan(lay[:, b, k]).all()
                    continue
                ko = where[tuple(np.round(tables.site_pos[b, k], 6))]
                worst = max(worst, float(np.abs(lay[:, b, k] - cc[:, b, ko]).max()) / scale)
    _say(f"TRI task-file run ({tables.n_pairs} pairs): chi at {len(ref)} cutoffs, worst error vs oracle {worst:.2e}")
    assert worst <= TOL
