"""Full-size parity against stored oracle results (tests/golden/*.npz).

The oracle takes minutes per right-hand side at the benchmark sizes, so its
results are written beforehand by tests/golden/make_full_size.py (oracle
only, on a CPU) and compared here with the library run on the same seeded
input:
  * one classical RK4 step (four right-hand sides) of the square J1-J2
    workload (range 7, 20 pairs, 32 frequencies) and of the honeycomb
    J1-J2-J3 workload (range 6, 14 pairs, 32 frequencies): the self-energy
    in full and 20000 sampled vertex elements;
  * one right-hand side of the pyrochlore workload (range 5, 31 pairs, 48
    frequencies): the self-energy flow and every element of 288 frequency
    triples, six in each t row.
FP64 bar: max |library - oracle| / max |oracle result| <= 1e-10.  FP32 mode
(vertex quadrature and lattice sums in FP32): the same comparison on the
increment (step result minus input, or the right-hand side) <= 1e-5.
"""

import os

import numpy as np
import pytest

import workloads as W
from tests.parity import pair_map

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-10
TOL_FP32 = 1e-5


def _say(*a):
    print(*a, flush=True)


def _setup(case, precision):
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    rec = np.load(os.path.join(GOLDEN, f"{case}.npz"))
    wl = W.workload(str(rec["workload"]))
    assert np.array_equal(wl.mesh, rec["mesh"])
    model = wl.model()
    tables = build_tables(model, wl.range)
    # the stored values are indexed by reduced pair: the tables must number
    # the pairs as when the file was written
    orc = oracle.Oracle(model, wl.range, wl.mesh)
    assert np.array_equal(pair_map(orc, tables), rec["pmap"]), "pair numbering changed since the file was written"
    ctx = Context(tables, wl.mesh, precision=precision)
    x = W.random_state(int(rec["nf"]), int(rec["ns"]), seed=int(rec["seed"]), scale=float(rec["scale"]))
    return rec, ctx, x


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["square_j1j2_rk4", "honeycomb_j123_rk4"])
def test_full_size_rk4_step(case, precision):
    import torch
    rec, ctx, x = _setup(case, precision)
    l0, l1 = (float(v) for v in rec["lam"])
    _say(f"full-size RK4 step {case} {precision}: {ctx.nf} frequencies, {ctx.ns} pairs, {l0} -> {l1}")
    xd = torch.from_numpy(x).cuda()
    ctx.step("rk4", l0, l1, xd)
    y = xd.cpu().numpy()
    nf, idx, val = ctx.nf, rec["index"], rec["value"]
    if precision == "fp64":
        scale = float(rec["scale_max"])
        err = max(np.abs(y[:nf] - rec["sigma"]).max(), np.abs(y[idx] - val).max()) / scale
        _say(f"  max error / max |state| = {err:.2e}")
        assert err <= TOL, err
    else:
        inc_ref = np.concatenate([rec["sigma"] - x[:nf], val - x[idx]])
        inc = np.concatenate([y[:nf] - x[:nf], y[idx] - x[idx]])
        err = np.abs(inc - inc_ref).max() / np.abs(inc_ref).max()
        _say(f"  max increment error / max |increment| = {err:.2e}")
        assert err <= TOL_FP32, err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_pyrochlore_rhs_triples(precision):
    import torch
    rec, ctx, x = _setup("pyrochlore_rhs", precision)
    lam = float(rec["lam"][0])
    tri = rec["triples"]
    assert len(set(int(t) for t in tri[:, 1])) == ctx.nf      # every t row
    _say(f"full-size pyrochlore RHS {precision}: {len(tri)} triples, lambda {lam}")
    d = ctx.rhs(lam, torch.from_numpy(x).cuda()).cpu().numpy()
    nf, ns = ctx.nf, ctx.ns
    n_su = nf * (nf + 1) // 2
    gs = d[nf:nf + n_su * nf * ns].reshape(n_su, nf, ns)
    gd = d[nf + n_su * nf * ns:].reshape(n_su, nf, ns)
    got = np.stack([np.stack([gs[a * (a + 1) // 2 + c, t], gd[a * (a + 1) // 2 + c, t]], axis=-1)
                    for a, t, c in tri])
    scale = float(rec["scale_max"])
    es = np.abs(d[:nf] - rec["sigma"]).max() / np.abs(rec["sigma"]).max()
    ev = np.abs(got - rec["value"]).max() / scale
    _say(f"  sigma {es:.2e}, vertex {ev:.2e}")
    assert es <= TOL, es          # the self-energy flow is FP64 in both modes
    assert ev <= (TOL if precision == "fp64" else TOL_FP32), ev


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lat,L", [("honeycomb", 8), ("square", 8)])
def test_partial_matrix_core_tiles_rhs_sampled(lat, L, precision):
    """23 (honeycomb range 8) and 25 (square range 8) pairs: the lattice-sum
    matrix padded to 24 and 28 rows, two 16x16 matrix-core tiles per side
    with partly filled second tiles (FP64), and the vector-ALU blocks (FP32);
    sampled triples against the oracle computed live."""
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    from tests.parity import compare_triples, expand_state
    params = dict(j1=1.0, j2=0.5, j3=0.25) if lat == "honeycomb" else dict(j1=1.0, j2=0.5)
    mesh = W.log_mesh(1e-2, 50.0, 12)
    model = W.model(lat, **params)
    tables = build_tables(model, L)
    assert tables.n_pairs == (23 if lat == "honeycomb" else 25)
    ctx = Context(tables, mesh, precision=precision)
    orc = oracle.Oracle(model, L, mesh)
    nf = ctx.nf
    x = W.random_state(nf, ctx.ns, seed=31, scale=0.2)
    lam = 0.29
    _say(f"partial tiles {lat} range {L} ({ctx.ns} pairs) {precision}")
    d = ctx.rhs(lam, torch.from_numpy(x).cuda()).cpu().numpy()
    xo = expand_state(orc, tables, x)
    dsig = orc.sigma_rhs(lam, xo)
    assert np.abs(dsig - d[:nf]).max() <= TOL * np.abs(dsig).max()
    rng = np.random.default_rng(3)
    tri = [(0, 0, 0), (nf - 1, nf - 1, nf - 1), (nf - 1, 0, 0)]
    for _ in range(9):
        a = int(rng.integers(nf)); c = int(rng.integers(a + 1)); t = int(rng.integers(nf))
        tri.append((a, t, c))
    ref = orc.vertex_rhs_triples(lam, xo, dsig, tri)
    err = compare_triples(orc, tables, tri, ref, d)
    _say(f"  vertex {err:.2e}")
    assert err <= (TOL if precision == "fp64" else TOL_FP32), err
