"""Batched flows (many lattices on one mesh, lockstep RK4) against the FP64
oracle, through the C ABI.

Per point the batch computes what a single flow computes; the tests check
each point against the oracle run on that point alone (FP64 bar 1e-10, FP32
bar 1e-5 per right-hand side), that the hipGraph replay of a step gives the
same bits as direct launches (several replays with other work in between),
that every launch shape gives the same bits, and that a diverging point
leaves the others untouched.
"""

import numpy as np
import pytest

import workloads as W
from tests.parity import compare_chi, compare_parts, compare_triples, expand_state

pytestmark = pytest.mark.gpu

MESH = W.log_mesh(1e-3, 100.0, 6)
# ragged pair counts 4, 9, 5, 7 (square range 2 and 4, honeycomb, pyrochlore)
POINTS = [("square", dict(j1=1.0), 2), ("square", dict(j1=1.0, j2=0.5), 4),
          ("honeycomb", dict(j1=0.6, j2=0.3, j3=0.45), 3), ("pyrochlore", dict(j1=1.0), 2)]


def _say(*a):
    print(*a, flush=True)


def _batch(points, mesh, precision):
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Batch
    models = [W.model(lat, **par) for lat, par, _ in points]
    tables = [build_tables(m, L) for m, (_, _, L) in zip(models, points)]
    b = Batch(tables, mesh, precision=precision)
    orcs = [oracle.Oracle(m, L, mesh, threads=0) for m, (_, _, L) in zip(models, points)]
    return torch, tables, b, orcs


def _random_batch_state(b, torch, seed, scale=1.0):
    parts = [W.random_state(b.nf, ns, seed=seed + p, scale=scale) for p, ns in enumerate(b.ns)]
    x = np.concatenate(parts)
    assert x.size == b.size
    return parts, torch.from_numpy(x).cuda()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("lam", [0.37, 4e-4, 170.0])
def test_batch_rhs_matches_oracle_per_point(precision, tol, lam):
    torch, tables, b, orcs = _batch(POINTS, MESH, precision)
    parts, x = _random_batch_state(b, torch, seed=11)
    d = b.rhs(lam, x).cpu().numpy()
    for p in range(b.n_points):
        ref = orcs[p].rhs(lam, expand_state(orcs[p], tables[p], parts[p]))
        es, ev = compare_parts(orcs[p], tables[p], ref, d[b.offsets[p]:b.offsets[p + 1]])
        _say(f"batch {precision} lam={lam} point {p} (ns={b.ns[p]}): sigma {es:.2e} vertex {ev:.2e}")
        assert es <= 1e-10 and ev <= tol


def test_batch_launch_shapes_give_identical_bits():
    torch, tables, b, orcs = _batch(POINTS, MESH, "fp32")
    _, x = _random_batch_state(b, torch, seed=3)
    ref = b.rhs(0.5, x).clone()
    for per in (1, 7, 32, 96, 512):
        for order in (0, 1):
            for split in (0, 1):
                b.set_launch(per, order, split)
                assert torch.equal(b.rhs(0.5, x), ref), (per, order, split)
    per, order, split = b.tune(0.5, x)
    _say(f"tuned launch: {per} workgroups per XCD, order {order}, split {split}")
    assert per in (32, 64, 96, 128, 192, 256, 384, 512) and order in (0, 1) and split in (0, 1)
    assert torch.equal(b.rhs(0.5, x), ref)


def test_batch_flow_graph_replays_match_direct_launches_and_oracle():
    torch, tables, b, orcs = _batch(POINTS[:3], MESH, "fp64")
    sched = W.geometric_schedule(50.0, 0.5, 12)
    x_direct = b.init_state()
    ok = b.flow(x_direct, sched, use_graph=False)
    assert all(ok)
    x_graph = b.init_state()
    assert all(b.flow(x_graph, sched, use_graph=True))
    assert torch.equal(x_graph, x_direct)
    # replay the captured step again, with other work and synchronisation in between
    for rep in range(2):
        b.rhs(0.7, x_direct)
        torch.cuda.synchronize()
        x_graph.copy_(b.init_state())
        assert all(b.flow(x_graph, sched, use_graph=True))
        assert torch.equal(x_graph, x_direct), rep
    xs = x_direct.cpu().numpy()
    for p in range(b.n_points):
        ref = orcs[p].flow(sched)
        es, ev = compare_parts(orcs[p], tables[p], ref, xs[b.offsets[p]:b.offsets[p + 1]])
        _say(f"batch flow point {p}: sigma {es:.2e} vertex {ev:.2e}")
        assert max(es, ev) <= 1e-10
    chis = b.chi(sched[-1], x_direct)
    for p in range(b.n_points):
        zz, dd = orcs[p].chi(sched[-1], orcs[p].flow(sched))
        assert compare_chi(orcs[p], tables[p], zz, dd, chis[p].cpu().numpy()) <= 1e-10


def test_batch_diverging_point_is_flagged_and_isolated():
    pts = [("square", dict(j1=1.0), 2), ("square", dict(j1=1e200), 2), ("honeycomb", dict(j1=0.5), 3)]
    torch, tables, b, orcs = _batch(pts, W.log_mesh(0.01, 10.0, 5), "fp64")
    sched = [5.0, 4.0, 3.0]
    x = b.init_state()
    ok = b.flow(x, sched, use_graph=True)
    assert ok == [True, False, True]
    xs = x.cpu().numpy()
    for p in (0, 2):
        ref = orcs[p].flow(sched)
        assert max(compare_parts(orcs[p], tables[p], ref, xs[b.offsets[p]:b.offsets[p + 1]])) <= 1e-10


def test_batch_scan_full_size_sampled():
    """The 64-point square J1-J2 scan (ranges 4..7, 24 frequencies) in FP32:
    one batch right-hand side, every element of sampled triples of one point
    of each range against the oracle."""
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Batch
    wl = W.workload("square_scan")
    pts = W.batch_scan_points(64)
    models = [W.model("square", j1=q["j1"], j2=q["j2"]) for q in pts]
    tables = [build_tables(m, q["range"]) for m, q in zip(models, pts)]
    b = Batch(tables, wl.mesh, precision="fp32")
    assert sorted(set(b.ns)) == [9, 12, 16, 20]
    parts = [W.random_state(b.nf, ns, seed=100 + p, scale=0.2) for p, ns in enumerate(b.ns)]
    x = torch.from_numpy(np.concatenate(parts)).cuda()
    lam = 0.3
    d = b.rhs(lam, x).cpu().numpy()
    nf = b.nf
    rng = np.random.default_rng(7)
    for p in (0, 1, 2, 63):
        orc = oracle.Oracle(models[p], pts[p]["range"], wl.mesh, threads=0)
        xo = expand_state(orc, tables[p], parts[p])
        dsig = orc.sigma_rhs(lam, xo)
        dp = d[b.offsets[p]:b.offsets[p + 1]]
        assert np.abs(dsig - dp[:nf]).max() <= 1e-10 * np.abs(dsig).max()
        tri = [(nf - 1, 0, 0), (nf - 1, nf // 2, nf - 1)]
        for _ in range(3):
            a = int(rng.integers(nf)); c = int(rng.integers(a + 1)); t = int(rng.integers(nf))
            tri.append((a, t, c))
        ref = orc.vertex_rhs_triples(lam, xo, dsig, tri)
        err = compare_triples(orc, tables[p], tri, ref, dp)
        _say(f"scan point {p} (range {pts[p]['range']}, ns={b.ns[p]}): vertex {err:.2e}")
        assert err <= 1e-5


def test_batch_with_single_pair_point():
    """A batch holding a range-0 point (the on-site pair only) beside larger
    ones: every point against its own oracle."""
    pts = [("square", dict(j1=1.0), 0)] + POINTS[:2]
    torch, tables, b, orcs = _batch(pts, MESH, "fp64")
    parts, x = _random_batch_state(b, torch, seed=17)
    d = b.rhs(0.3, x).cpu().numpy()
    for p in range(b.n_points):
        ref = orcs[p].rhs(0.3, expand_state(orcs[p], tables[p], parts[p]))
        es, ev = compare_parts(orcs[p], tables[p], ref, d[b.offsets[p]:b.offsets[p + 1]])
        assert es <= 1e-10 and ev <= 1e-10, (p, es, ev)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_batch_with_non_adjacent_exchange_partners(precision, tol):
    """Honeycomb range 6 (14 pairs) beside square points in one batch: its
    pairs include exchange partners that are not adjacent (in FP32 the case
    where a lane's two pairs need two loads per corner).  Every element of
    each point against a single context of the same precision (pinned to the
    oracle at full size by the FP32 and FP64 parity tests)."""
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Batch, Context
    mesh = W.log_mesh(1e-3, 100.0, 8)
    models = [W.model("honeycomb", j1=0.6, j2=0.3, j3=0.45), W.model("square", j1=1.0, j2=0.5)]
    tables = [build_tables(models[0], 6), build_tables(models[1], 3)]
    b = Batch(tables, mesh, precision=precision)
    parts, x = _random_batch_state(b, torch, seed=21, scale=0.3)
    lam = 0.29
    d = b.rhs(lam, x).cpu().numpy()
    for p, t in enumerate(tables):
        c = Context(t, mesh, precision=precision)
        ref = c.rhs(lam, torch.from_numpy(parts[p]).cuda()).cpu().numpy()
        got = d[b.offsets[p]:b.offsets[p + 1]]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        _say(f"batch {precision} point {p} (ns={b.ns[p]}) vs single context: {err:.2e}")
        assert err <= tol, err
