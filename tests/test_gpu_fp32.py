"""FP32 mode against the FP64 oracle, through the C ABI.

In FP32 mode the vertex interpolation, the channel products, the quadrature
sums and the lattice-sum matrix run in single precision (per-chunk partial
sums folded with compensated summation); the self-energy flow, the node
tables, the state, the Runge-Kutta steps and chi stay FP64.  Tolerances:

* self-energy derivative: the FP64 bar, 1e-10 of its own max norm;
* vertex derivative: TOL_RHS = 1e-5 of its max norm per right-hand side;
* chi after a whole flow: TOL_CHI = 1e-4 of max |chi|.

Each test prints the measured errors.
"""

import math
import zlib

import numpy as np
import pytest

import workloads as W
from tests.parity import compare_chi, compare_parts, compare_triples, expand_state

pytestmark = pytest.mark.gpu

TOL_SIGMA = 1e-10
TOL_RHS = 1e-5
TOL_CHI = 1e-4

CASES = {
    "square_L2_N8": ("square", dict(j1=1.0), 2, W.log_mesh(0.005, 50.0, 8)),
    "square_j1j2_L3_N7": ("square", dict(j1=1.0, j2=0.5), 3, W.log_mesh(1e-3, 100.0, 7)),
    "honeycomb_L3_N6": ("honeycomb", dict(j1=0.6, j2=0.3, j3=0.45), 3, W.log_mesh(1e-3, 100.0, 6)),
    "pyrochlore_L2_N5": ("pyrochlore", dict(j1=1.0), 2, W.log_mesh(1e-3, 100.0, 5)),
}


def _setup(name, precision="fp32"):
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    lat, params, L, mesh = CASES[name]
    model = W.model(lat, **params)
    tables = build_tables(model, L)
    ctx = Context(tables, mesh, precision=precision)
    orc = oracle.Oracle(model, L, mesh, threads=0)
    return torch, tables, ctx, orc


def _say(*a):
    print(*a, flush=True)


def _seed(*key) -> int:
    """A seed fixed by the case name (the same in every process, unlike hash())."""
    return zlib.crc32("/".join(map(str, key)).encode()) % 1000


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("lam_kind", ["low", "mid", "mesh", "high"])
def test_fp32_rhs_random_state(name, lam_kind):
    torch, tables, ctx, orc = _setup(name)
    mesh = ctx.mesh
    lam = {"low": 0.5 * mesh[0], "mid": 0.37, "mesh": float(mesh[len(mesh) // 2]),
           "high": 1.7 * mesh[-1]}[lam_kind]
    x = W.random_state(ctx.nf, ctx.ns, seed=_seed(name, lam_kind))
    d = ctx.rhs(lam, torch.from_numpy(x).cuda()).cpu().numpy()
    ref = orc.rhs(lam, expand_state(orc, tables, x))
    es, ev = compare_parts(orc, tables, ref, d)
    _say(f"fp32 rhs {name} lam={lam:.4g}: sigma {es:.2e} vertex {ev:.2e}")
    assert es <= TOL_SIGMA, es
    assert ev <= TOL_RHS, ev


@pytest.mark.parametrize("which", ["square_j1j2", "honeycomb_j123", "pyrochlore"])
def test_fp32_full_size_rhs_sampled(which):
    """FP32 at the full workload sizes: every element of a sample of triples
    against the oracle, and every element against the FP64 kernels (which
    the FP64 tests pin to the oracle).  Honeycomb (14 pairs) and pyrochlore
    (31 pairs, an odd count) have pairs whose exchange partners are not
    adjacent, the case where a lane's two pairs need two loads per corner."""
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    wl = W.workload(which)
    model = wl.model()
    tables = build_tables(model, wl.range)
    ctx = Context(tables, wl.mesh, precision="fp32")
    orc = oracle.Oracle(model, wl.range, wl.mesh, threads=0)
    nf = ctx.nf
    x = W.random_state(nf, ctx.ns, seed=5, scale=0.2)
    lam = 0.21
    d = ctx.rhs(lam, torch.from_numpy(x).cuda()).cpu().numpy()
    d64 = Context(tables, wl.mesh).rhs(lam, torch.from_numpy(x).cuda()).cpu().numpy()
    e64 = np.abs(d[nf:] - d64[nf:]).max() / np.abs(d64[nf:]).max()
    _say(f"fp32 {which} whole vertex vs fp64 kernels: {e64:.2e}")
    assert e64 <= TOL_RHS, e64
    xo = expand_state(orc, tables, x)
    dsig = orc.sigma_rhs(lam, xo)
    assert np.abs(dsig - d[:nf]).max() <= TOL_SIGMA * np.abs(dsig).max()
    rng = np.random.default_rng(2)
    tri = [(0, 0, 0), (nf - 1, nf - 1, nf - 1), (nf - 1, 0, 0), (nf - 1, nf // 2, nf - 1)]
    for _ in range(8):
        a = int(rng.integers(nf)); c = int(rng.integers(a + 1)); t = int(rng.integers(nf))
        tri.append((a, t, c))
    ref = orc.vertex_rhs_triples(lam, xo, dsig, tri)
    err = compare_triples(orc, tables, tri, ref, d)
    _say(f"fp32 {which} full-size sampled vertex error {err:.2e}")
    assert err <= TOL_RHS, err


def test_fp32_rk4_flow_chi():
    """The small square workload (range 2, 8 frequencies, RK4 50 -> 0.5 in
    40 steps) in FP32 mode against the FP64 oracle flow: chi_ij at every
    step and chi(k) at the end."""
    torch, tables, ctx, orc = _setup("square_L2_N8")
    wl = W.workload("square_tiny")
    x = ctx.init_state()
    got = []
    ctx.flow(x, schedule=wl.schedule, scheme="rk4",
             observer=lambda lam, chi, ck: got.append((lam, chi.cpu().numpy().copy())) and 0)
    ref_chi = []
    xo = orc.flow(wl.schedule, observer=lambda lam, xs: ref_chi.append((lam, orc.chi(lam, xs))))
    es, ev = compare_parts(orc, tables, xo, x.cpu().numpy())
    worst = 0.0
    for (lg, cg), (lr, (zz, dd)) in zip(got, ref_chi):
        assert lg == lr
        worst = max(worst, compare_chi(orc, tables, zz, dd, cg))
    zz, dd = ref_chi[-1][1]
    kp = np.array([[math.pi, math.pi, 0.0], [0.0, 0.0, 0.0], [math.pi, 0.0, 0.0]])
    ck = ctx.chi_k(torch.from_numpy(got[-1][1].reshape(-1)).cuda(), torch.from_numpy(kp).cuda()).cpu().numpy()
    ref_k = orc.chi_k(zz, kp)
    ek = float(np.abs(ck - ref_k).max() / np.abs(ref_k).max())
    _say(f"fp32 flow: final state sigma {es:.2e} vertex {ev:.2e}; chi worst step {worst:.2e}; chi(k) {ek:.2e}")
    assert worst <= TOL_CHI and ek <= TOL_CHI
    assert ev <= 1e-4


def test_fp32_and_fp64_contexts_coexist():
    """Two contexts of different precision on one lattice give the same
    self-energy derivative (FP64 in both) and vertex derivatives within the
    FP32 tolerance of each other's oracle error."""
    torch, tables, c32, orc = _setup("honeycomb_L3_N6")
    _, _, c64, _ = _setup("honeycomb_L3_N6", precision="fp64")
    x = torch.from_numpy(W.random_state(c32.nf, c32.ns, seed=9)).cuda()
    d32 = c32.rhs(0.3, x).cpu().numpy()
    d64 = c64.rhs(0.3, x).cpu().numpy()
    assert np.array_equal(d32[:c32.nf], d64[:c64.nf])
    ref = orc.rhs(0.3, expand_state(orc, tables, x.cpu().numpy()))
    assert compare_parts(orc, tables, ref, d64)[1] <= 1e-10
    assert compare_parts(orc, tables, ref, d32)[1] <= TOL_RHS
