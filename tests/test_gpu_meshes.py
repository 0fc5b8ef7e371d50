"""Meshes with clusters of points, against the FP64 oracle through the C ABI.

The vertex kernels bracket a frequency through a per-mesh look-up table
(buckets of a fixed fraction of an octave, about 0.03 wide at w = 1.5 here)
and a forward search from the bucket's first bracket; on the logarithmic
meshes of the other tests that search takes at most one step.  These meshes
put clusters of points 1e-4 apart inside one bucket, in the middle and at
both ends of a logarithmic mesh, so that arguments in those buckets step over
several points (and, at the ends, reach the last bracket).  Bars as
elsewhere: FP64 right-hand side 1e-10, FP32 1e-5 (self-energy 1e-10), a
batch per point 1e-10, and the reverse-mode kernels by <v, J u> =
<J^T v, u> with the oracle's J u to 1e-9.
"""

import numpy as np
import pytest

import workloads as W
from tests.parity import compare_parts, expand_state, restrict_state

pytestmark = pytest.mark.gpu

BASE = list(W.log_mesh(0.05, 20.0, 7))
MESHES = {
    "middle": np.array(sorted(BASE + [1.5, 1.5001, 1.5002, 1.5003])),
    "ends": np.array(sorted(BASE + [0.050001, 0.050002, 19.9998, 19.9999])),
}
# cutoffs: generic, inside the middle cluster, near the top cluster
LAMS = (0.3, 1.50015, 9.99995)


def _say(*a):
    print(*a, flush=True)


def _setup(mesh, precision="fp64", lat="square", params=None, L=2):
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    model = W.model(lat, **(params or dict(j1=1.0, j2=0.5)))
    tables = build_tables(model, L)
    return tables, Context(tables, mesh, precision=precision), oracle.Oracle(model, L, mesh, threads=0)


def test_mesh_lookup_hits_the_clusters():
    """The buckets of the clustered points hold several points each (so the
    search steps over them), computed with the kernels' own key."""
    for name, mesh in MESHES.items():
        shift = 32
        key = lambda v, s: int(np.float64(v).view(np.uint64)) >> s
        while key(mesh[-1], shift) - key(mesh[0], shift) >= 512:
            shift += 1
        keys = [key(v, shift) for v in mesh]
        most = max(keys.count(k) for k in keys)
        _say(f"{name}: shift {shift}, at most {most} mesh points per bucket")
        assert most >= 2


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_rhs_on_clustered_meshes(name, precision, tol):
    import torch
    mesh = MESHES[name]
    tables, ctx, orc = _setup(mesh, precision)
    x = W.random_state(ctx.nf, ctx.ns, seed=41, scale=0.5)
    xo = expand_state(orc, tables, x)
    for lam in LAMS:
        d = ctx.rhs(lam, torch.from_numpy(x).cuda()).cpu().numpy()
        es, ev = compare_parts(orc, tables, orc.rhs(lam, xo), d)
        _say(f"{name} {precision} lam={lam}: sigma {es:.2e} vertex {ev:.2e}")
        assert es <= 1e-10 and ev <= tol


def test_batch_on_a_clustered_mesh():
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Batch
    mesh = MESHES["middle"]
    pts = [("square", dict(j1=1.0, j2=0.5), 2), ("honeycomb", dict(j1=0.6, j2=0.3, j3=0.45), 2)]
    models = [W.model(lat, **par) for lat, par, _ in pts]
    tables = [build_tables(m, L) for m, (_, _, L) in zip(models, pts)]
    b = Batch(tables, mesh, precision="fp64")
    parts = [W.random_state(b.nf, ns, seed=50 + p, scale=0.5) for p, ns in enumerate(b.ns)]
    d = b.rhs(1.50015, torch.from_numpy(np.concatenate(parts)).cuda()).cpu().numpy()
    for p, (m, (_, _, L)) in enumerate(zip(models, pts)):
        orc = oracle.Oracle(m, L, mesh, threads=0)
        ref = orc.rhs(1.50015, expand_state(orc, tables[p], parts[p]))
        es, ev = compare_parts(orc, tables[p], ref, d[b.offsets[p]:b.offsets[p + 1]])
        _say(f"batch point {p}: sigma {es:.2e} vertex {ev:.2e}")
        assert es <= 1e-10 and ev <= 1e-10


def test_reverse_mode_on_a_clustered_mesh():
    import torch
    mesh = MESHES["middle"]
    tables, ctx, orc = _setup(mesh)
    nf = ctx.nf
    x = W.random_state(nf, ctx.ns, seed=60, scale=0.3)
    rng = np.random.default_rng(61)
    u = W.random_state(nf, ctx.ns, seed=62, scale=1.0)
    u[:nf] = 0.0                       # a vertex direction: the five-point stencil is exact
    f = lambda xr: restrict_state(orc, tables, orc.rhs(1.50015, expand_state(orc, tables, xr)))
    ju = sum(c * f(x + s * u) for s, c in ((-2, 1 / 12), (-1, -8 / 12), (1, 8 / 12), (2, -1 / 12)))
    v = rng.standard_normal(x.size)
    g = ctx.rhs_vjp(1.50015, torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda()).cpu().numpy()
    lhs, rhs = float(v @ ju), float(g @ u)
    err = abs(lhs - rhs) / max(abs(lhs), np.abs(g).max() * np.abs(u).max())
    _say(f"clustered mesh: <v,Ju>={lhs:.12e} <J^T v,u>={rhs:.12e} rel {err:.2e}")
    assert err <= 1e-9
