"""Flow checkpoints through the C ABI (pffrg_flow_position and the resume
fields of pffrg_flow_opts) on the GPU.

A flow stopped after some accepted steps and resumed from its snapshot, with
a fresh state tensor, ends bitwise where the uninterrupted flow ends and
after the same number of steps: adaptive (DOPRI54, FP64 and FP32) and fixed
RK4 schedules.  A finished fixed-schedule flow extended to a longer schedule
equals the direct flow bitwise; a finished adaptive flow extended to a lower
cutoff continues to it.  A snapshot of another calculation is refused and
force_restart ignores a snapshot.  A batch flow run in segments and
checkpointed, then extended from its snapshot to a longer schedule, equals
the one-call batch flow bitwise, diverging point included; so does the
batch breakdown scan, which steps one RK4 step at a time.

Breakdown detector on full flows (square J1-J2, range 7, 32 frequencies,
adaptive 100 -> 0.01, chi(k) on 64 x 64 points): the ordered phases at
J2/J1 = 0 (Neel) and 1 (stripe) break down at a kink between Lambda = 0.3
and 0.7, J2/J1 = 0.5 flows smoothly (a regression check of the heuristic;
parity unpinned: the paper fixes no criterion).
"""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

MESH = W.log_mesh(0.005, 50.0, 8)
ADAPT = dict(scheme="dopri54", lam_start=20.0, lam_stop=0.05, rtol=1e-6, atol=1e-9, h0=0.05, hmin=1e-9)
SCHED = list(20.0 * 0.85 ** np.arange(38))        # 20 -> 0.0095


def _say(*a):
    print(*a, flush=True)


def _ctx(j2=0.5, precision="fp64"):
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    return Context(build_tables(W.model("square", j1=1.0, j2=j2), 2), MESH, precision=precision)


class _StopAfter:
    def __init__(self, n):
        self.n, self.k = n, 0

    def __call__(self, lam, chi, chik):
        self.k += 1
        return self.k >= self.n


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adaptive_flow_resumes_bitwise(tmp_path, precision):
    import torch
    from paper_2109_13317_amd import checkpoint as C
    ctx = _ctx(precision=precision)
    x_ref = ctx.init_state()
    n_ref = ctx.flow(x_ref, **ADAPT)
    p = str(tmp_path / "a.checkpoint")
    x = ctx.init_state()
    n1 = C.flow(ctx, x, p, every=0.0, observer=_StopAfter(7), **ADAPT)
    assert n1 == 7 and C.read(p).meta["status"] == "running"
    x2 = ctx.init_state()
    n2 = C.flow(ctx, x2, p, every=0.0, **ADAPT)
    meta = C.read(p).meta
    _say(f"{precision}: uninterrupted {n_ref} steps, resumed {n1} + {n2}, status {meta['status']}")
    assert meta["status"] == "finished" and meta["steps"] == n_ref == n1 + n2
    assert torch.equal(x2, x_ref)
    assert float.fromhex(meta["lambda"]) == pytest.approx(0.05, rel=1e-12)
    assert C.flow(ctx, x2, p, **ADAPT) == 0 and torch.equal(x2, x_ref)      # nothing left to do


def test_fixed_schedule_resumes_and_extends_bitwise(tmp_path):
    import torch
    from paper_2109_13317_amd import checkpoint as C
    ctx = _ctx()
    x_ref = ctx.init_state()
    assert ctx.flow(x_ref, scheme="rk4", schedule=SCHED) == len(SCHED) - 1
    p = str(tmp_path / "f.checkpoint")
    x = ctx.init_state()
    assert C.flow(ctx, x, p, scheme="rk4", schedule=SCHED[:20], every=0.0, observer=_StopAfter(5)) == 5
    assert C.read(p).meta["ladder"] == 5
    # resume the first 20 cutoffs, then extend to the whole schedule
    assert C.flow(ctx, x, p, scheme="rk4", schedule=SCHED[:20], every=1e9) == 14
    assert C.read(p).meta["status"] == "finished"
    x2 = ctx.init_state()
    assert C.flow(ctx, x2, p, scheme="rk4", schedule=SCHED, every=1e9) == len(SCHED) - 20
    meta = C.read(p).meta
    assert meta["status"] == "finished" and meta["steps"] == len(SCHED) - 1
    assert torch.equal(x2, x_ref)


def test_finished_adaptive_flow_extends_to_a_lower_cutoff(tmp_path):
    from paper_2109_13317_amd import checkpoint as C
    ctx = _ctx()
    p = str(tmp_path / "e.checkpoint")
    x = ctx.init_state()
    n1 = C.flow(ctx, x, p, **dict(ADAPT, lam_stop=0.5))
    assert C.read(p).meta["status"] == "finished"
    n2 = C.flow(ctx, x, p, **ADAPT)
    meta = C.read(p).meta
    assert n2 > 0 and meta["status"] == "finished" and meta["steps"] == n1 + n2
    assert float.fromhex(meta["lambda"]) == pytest.approx(0.05, rel=1e-12)
    x_ref = ctx.init_state()
    ctx.flow(x_ref, **ADAPT)
    xa, xr = x.cpu().numpy(), x_ref.cpu().numpy()
    err = np.abs(xa - xr).max() / np.abs(xr).max()
    _say(f"extended flow vs direct flow: {err:.2e}")
    assert np.isfinite(xa).all() and err < 1e-4


def test_snapshot_of_another_calculation_is_refused(tmp_path):
    import torch
    from paper_2109_13317_amd import checkpoint as C
    p = str(tmp_path / "o.checkpoint")
    ctx = _ctx(j2=0.5)
    C.flow(ctx, ctx.init_state(), p, every=0.0, observer=_StopAfter(3), **ADAPT)
    other = _ctx(j2=0.0)
    with pytest.raises(ValueError, match="another calculation"):
        C.flow(other, other.init_state(), p, **ADAPT)
    x_ref = ctx.init_state()
    ctx.flow(x_ref, **ADAPT)
    x = ctx.init_state()
    C.flow(ctx, x, p, force_restart=True, **ADAPT)          # ignores the running snapshot
    assert torch.equal(x, x_ref)


def test_position_before_any_step_is_an_error():
    from paper_2109_13317_amd._lib import PffrgError
    ctx = _ctx()
    with pytest.raises(PffrgError):
        ctx.position()
    x = ctx.init_state()
    ctx.flow(x, scheme="rk4", schedule=SCHED[:4])
    lam, ll, lad = ctx.position()
    assert lam == SCHED[3] and lad == 3 and ll == pytest.approx(np.log(SCHED[3]), rel=1e-15)


@pytest.mark.parametrize("j2,kind,lo,hi", [(0.0, "kink", 0.4, 0.7), (0.5, None, None, None),
                                           (1.0, "kink", 0.3, 0.5)])
def test_breakdown_marks_the_ordered_phases(j2, kind, lo, hi):
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.breakdown import ChiMaxRecorder
    from paper_2109_13317_amd.flow import Context
    wl = W.workload("square_j1j2")
    ctx = Context(build_tables(W.model("square", j1=1.0, j2=j2), 7), wl.mesh)
    g = 2 * np.pi * (np.arange(64) / 64 - 0.5)
    kx, ky = np.meshgrid(g, g, indexing="ij")
    kp = torch.from_numpy(np.stack([kx.ravel(), ky.ravel(), np.zeros(kx.size)], 1).copy()).cuda()
    rec = ChiMaxRecorder()
    x = ctx.init_state()
    ctx.flow(x, scheme="dopri54", lam_start=100.0, lam_stop=0.01, rtol=1e-4, atol=1e-6, h0=0.05, hmin=1e-9,
             kpoints=kp, observer=rec)
    b = rec.breakdown(lam_max=wl.mesh[-1] / 4)
    _say(f"J2/J1 = {j2}: {len(rec.lams)} steps, breakdown {b.kind} at Lambda = {b.lam}")
    assert b.kind == kind
    if kind is not None:
        assert lo < b.lam < hi


def test_batch_flow_checkpoints_and_extends_bitwise(tmp_path):
    import torch
    from paper_2109_13317_amd import build_tables, checkpoint as C
    from paper_2109_13317_amd.flow import Batch
    pts = [("square", dict(j1=1.0, j2=0.5), 2), ("square", dict(j1=1e200), 2),
           ("honeycomb", dict(j1=0.6, j2=0.3, j3=0.45), 2)]
    tables = [build_tables(W.model(lat, **par), L) for lat, par, L in pts]
    b = Batch(tables, W.log_mesh(1e-3, 100.0, 6), precision="fp64")
    sched = list(50.0 * 0.8 ** np.arange(13))
    x_ref = b.init_state()
    ok_ref = b.flow(x_ref, sched)
    assert ok_ref == [True, False, True]
    p = str(tmp_path / "b.checkpoint")
    x = b.init_state()
    assert C.batch_flow(b, x, p, sched[:7], every=0.0, segment=4) == ok_ref
    meta = C.read(p).meta
    assert meta["status"] == "finished" and meta["index"] == 6 and meta["steps"] == 6
    x2 = b.init_state()
    assert C.batch_flow(b, x2, p, sched, every=0.0, segment=5) == ok_ref
    meta = C.read(p).meta
    assert meta["index"] == len(sched) - 1 and meta["steps"] == len(sched) - 1
    assert torch.equal(torch.nan_to_num(x2, nan=7.0), torch.nan_to_num(x_ref, nan=7.0))
    with pytest.raises(ValueError, match="another calculation"):
        C.batch_flow(Batch(tables[:2], W.log_mesh(1e-3, 100.0, 6), precision="fp64"),
                     b.init_state()[:0], p, sched)


def test_batch_breakdowns_steps_like_one_flow_call():
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.breakdown import batch_breakdowns
    from paper_2109_13317_amd.flow import Batch
    pts = [("square", dict(j1=1.0, j2=0.5), 3), ("square", dict(j1=1e200), 2)]
    tables = [build_tables(W.model(lat, **par), L) for lat, par, L in pts]
    b = Batch(tables, W.log_mesh(1e-3, 100.0, 8), precision="fp64")
    sched = list(50.0 * 0.8 ** np.arange(15))
    x_ref = b.init_state()
    b.flow(x_ref, sched)
    g = 2 * np.pi * (np.arange(8) / 8 - 0.5)
    kx, ky = np.meshgrid(g, g, indexing="ij")
    kp = torch.from_numpy(np.stack([kx.ravel(), ky.ravel(), np.zeros(kx.size)], 1).copy()).cuda()
    x = b.init_state()
    bds, lams, chi_max = batch_breakdowns(b, x, sched, kp)
    assert torch.equal(torch.nan_to_num(x, nan=7.0), torch.nan_to_num(x_ref, nan=7.0))
    assert lams == sched[1:] and chi_max.shape == (2, len(sched) - 1)
    assert np.isfinite(chi_max[0]).all() and (chi_max[0] > 0).all()
    assert bds[1].kind == "nonfinite"
    _say(f"batch breakdowns: {[(d.kind, d.lam) for d in bds]}")
