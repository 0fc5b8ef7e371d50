"""Host parts of flow checkpoints and the breakdown detector (no GPU).

Snapshots: exact round trip of state and record, atomic replacement, and the
identity checks that keep a snapshot from continuing another calculation.
Breakdown detector (a heuristic, parity unpinned: the paper names the
signatures, divergence or kink of chi_max(Lambda), but fixes no criterion):
smooth curves stay unflagged on fixed and irregular step sequences; a pole,
a steep power law, a slope jump, a peak and a non-finite value are flagged
where they are.
"""

import os
from types import SimpleNamespace

import numpy as np
import pytest

import workloads as W
from paper_2109_13317_amd import build_tables
from paper_2109_13317_amd import breakdown as B
from paper_2109_13317_amd import checkpoint as C


def _fake_ctx(j2=0.5, mesh=None, precision="fp64"):
    t = build_tables(W.model("square", j1=1.0, j2=j2), 2)
    mesh = W.log_mesh(0.005, 50.0, 8) if mesh is None else mesh
    nf = len(mesh)
    size = nf + 2 * nf * (nf + 1) // 2 * nf * t.n_pairs
    return SimpleNamespace(mesh=np.asarray(mesh, dtype=np.float64), tables=t, precision=precision, size=size)


def test_snapshot_round_trip_is_exact_and_atomic(tmp_path):
    rng = np.random.default_rng(5)
    state = rng.standard_normal(1001) * 10.0 ** rng.integers(-300, 300, 1001)
    meta = dict(C.identity(_fake_ctx(), "dopri54", rtol=1e-6, atol=1e-10, h0=0.05, hmin=1e-8),
                status="running", log_lambda=(-1.2345678901234567).hex(), ladder=-7, steps=12)
    p = str(tmp_path / "flow.checkpoint")
    C.write(p, state, meta)
    assert not os.path.exists(p + ".tmp")
    snap = C.read(p)
    assert snap.state.tobytes() == state.tobytes()
    assert snap.meta == meta
    assert float.fromhex(snap.meta["log_lambda"]) == -1.2345678901234567
    # overwrite: the new snapshot replaces the old one whole
    C.write(p, state[:10], dict(meta, status="finished"))
    snap = C.read(p)
    assert snap.state.size == 10 and snap.meta["status"] == "finished"


def test_snapshot_with_unknown_format_is_refused(tmp_path):
    p = str(tmp_path / "x.checkpoint")
    C.write(p, np.zeros(3), {"format": 99})
    with pytest.raises(ValueError, match="format"):
        C.read(p)


def test_identity_tells_calculations_apart():
    base = C.identity(_fake_ctx(), "dopri54", rtol=1e-6, atol=1e-10, h0=0.05, hmin=1e-8)
    C._check_identity(base, base, "p")
    others = [
        C.identity(_fake_ctx(j2=0.25), "dopri54", rtol=1e-6, atol=1e-10, h0=0.05, hmin=1e-8),
        C.identity(_fake_ctx(mesh=W.log_mesh(0.005, 50.0, 9)), "dopri54", rtol=1e-6, atol=1e-10, h0=0.05,
                   hmin=1e-8),
        C.identity(_fake_ctx(precision="fp32"), "dopri54", rtol=1e-6, atol=1e-10, h0=0.05, hmin=1e-8),
        C.identity(_fake_ctx(), "dopri54", rtol=1e-7, atol=1e-10, h0=0.05, hmin=1e-8),
    ]
    for o in others:
        with pytest.raises(ValueError, match="another calculation"):
            C._check_identity(base, o, "p")
    assert C.lattice_digest(_fake_ctx().tables) != C.lattice_digest(_fake_ctx(j2=0.25).tables)


def test_fixed_schedule_may_only_be_extended():
    sched = list(50.0 * 0.9 ** np.arange(30))
    ctx = _fake_ctx()
    saved = C.identity(ctx, "rk4", schedule=sched[:12])
    C._check_identity(saved, C.identity(ctx, "rk4", schedule=sched), "p")          # longer: fine
    moved = list(sched)
    moved[5] *= 1.0 + 1e-15
    with pytest.raises(ValueError, match="schedule"):
        C._check_identity(saved, C.identity(ctx, "rk4", schedule=moved), "p")


GEOM = 50.0 * 0.95 ** np.arange(260)        # 50 -> ~0.08, the bench's RK4 ratio


def test_smooth_flows_are_not_flagged():
    assert B.find_breakdown(GEOM, 1.0 / (GEOM + 0.2)).kind is None
    assert B.find_breakdown(GEOM, 2.0 + GEOM ** -0.5).kind is None
    rng = np.random.default_rng(3)
    lam = 100.0 * np.cumprod(rng.uniform(0.5, 0.98, 120))                   # irregular adaptive steps
    assert B.find_breakdown(lam, 1.0 / (lam + 0.2)).kind is None


def test_pole_is_flagged_just_above_it():
    lam = GEOM[GEOM > 0.3001]
    b = B.find_breakdown(lam, 1.0 / (lam - 0.3))
    assert b.kind in ("divergence", "kink") and 0.3 < b.lam < 0.4


def test_steep_growth_is_a_divergence():
    b = B.find_breakdown(GEOM, GEOM ** -10.0)
    assert b.kind == "divergence" and b.index == 1


def test_slope_jump_is_a_kink_at_the_jump():
    t = np.log(GEOM)
    tc = np.log(0.5)
    y = np.where(t > tc, -0.5 * t, -0.5 * tc - 3.0 * (t - tc))
    b = B.find_breakdown(GEOM, np.exp(y))
    assert b.kind == "kink" and 0.45 < b.lam <= 0.5


def test_peak_is_a_kink():
    t = np.log(GEOM)
    tc = np.log(0.4)
    y = np.where(t > tc, -t, -tc + 2.0 * (t - tc))
    b = B.find_breakdown(GEOM, np.exp(y))
    assert b.kind == "kink" and 0.36 < b.lam <= 0.4


def test_steps_above_lam_max_are_skipped():
    chi = 1.0 / (GEOM + 0.2)
    chi[:4] = [1e-6, 1e-4, 1e-3, 3e-3]                  # a steep start at the mesh edge
    assert B.find_breakdown(GEOM, chi).index in (1, 2)
    assert B.find_breakdown(GEOM, chi, lam_max=GEOM[4]).kind is None


def test_non_finite_is_flagged_where_it_appears():
    chi = 1.0 / (GEOM + 0.2)
    chi[77] = np.nan
    b = B.find_breakdown(GEOM, chi)
    assert b.kind == "nonfinite" and b.index == 77
    with pytest.raises(ValueError):
        B.find_breakdown(GEOM, chi[:-1])


def test_recorder_takes_the_maximum():
    import torch
    rec = B.ChiMaxRecorder()
    rec(2.0, torch.tensor([[1.0, 3.0], [9.0, 9.0]]), None)
    rec(1.0, torch.tensor([[1.0, 3.0], [9.0, 9.0]]), torch.tensor([0.5, 4.0, 2.0]))
    assert rec.lams == [2.0, 1.0] and rec.chi_max == [3.0, 4.0]
    assert rec.breakdown().kind is None
