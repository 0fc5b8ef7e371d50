"""GPU parity: the HIP library against the FP64 oracle, through the C ABI.

Bar (FP64): max |gpu - oracle| / max |oracle| <= 1e-10 over every element
(the oracle's unreduced elements, matched to the library's reduced pairs by
site position).  Sizes span several workgroups per launch and the lattices
with non-trivial pair exchange (honeycomb, pyrochlore).
"""

import math
import zlib

import numpy as np
import pytest

import workloads as W
from tests.parity import compare_chi_sites, compare_chi, compare_triples, compare_vertex, expand_state

pytestmark = pytest.mark.gpu

TOL = 1e-10

CASES = {
    # name: (lattice, params, range, mesh)
    "square_L2_N8": ("square", dict(j1=1.0), 2, W.log_mesh(0.005, 50.0, 8)),
    "square_j1j2_L3_N7": ("square", dict(j1=1.0, j2=0.5), 3, W.log_mesh(1e-3, 100.0, 7)),
    "honeycomb_L3_N6": ("honeycomb", dict(j1=0.6, j2=0.3, j3=0.45), 3, W.log_mesh(1e-3, 100.0, 6)),
    "pyrochlore_L2_N5": ("pyrochlore", dict(j1=1.0), 2, W.log_mesh(1e-3, 100.0, 5)),
}


def _setup(name):
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    lat, params, L, mesh = CASES[name]
    model = W.model(lat, **params)
    tables = build_tables(model, L)
    ctx = Context(tables, mesh)
    orc = oracle.Oracle(model, L, mesh, threads=0)
    return torch, tables, ctx, orc


def _say(*a):
    print(*a, flush=True)


def _seed(*key) -> int:
    """A seed fixed by the case name (the same in every process, unlike hash())."""
    return zlib.crc32("/".join(map(str, key)).encode()) % 1000


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("lam_kind", ["low", "mid", "mesh", "half", "high"])
def test_rhs_random_state(name, lam_kind):
    """'half' puts Lambda at half a mesh frequency, so transfer frequencies
    2 Lambda sit on the mesh and delta-point propagators meet |w| = Lambda
    exactly (the theta = 1/2 ties)."""
    torch, tables, ctx, orc = _setup(name)
    mesh = ctx.mesh
    lam = {"low": 0.5 * mesh[0], "mid": 0.37, "mesh": float(mesh[len(mesh) // 2]),
           "half": 0.5 * float(mesh[len(mesh) // 2]), "high": 1.7 * mesh[-1]}[lam_kind]
    x = W.random_state(ctx.nf, ctx.ns, seed=_seed(name, lam_kind))
    _say(f"rhs {name} lam={lam}")
    d = ctx.rhs(lam, torch.from_numpy(x).cuda()).cpu().numpy()
    ref = orc.rhs(lam, expand_state(orc, tables, x))
    err = compare_vertex(orc, tables, ref, d)
    assert err <= TOL, err


# beyond 20 pairs: the FP64 lattice sum on two matrix-core tiles per side
# (24, 28 and 32 rows), the FP32 one on vector-ALU blocks, and the
# contraction with the tabulated terms in lane runs split on the host
BEYOND_20 = {
    "honeycomb_L8_N4": ("honeycomb", dict(j1=1.0, j2=0.5, j3=0.25), 8, W.log_mesh(1e-2, 50.0, 4)),   # 23 pairs
    "square_L8_N4": ("square", dict(j1=1.0, j2=0.5), 8, W.log_mesh(1e-2, 50.0, 4)),                   # 25 pairs
    "pyrochlore_L5_N3": ("pyrochlore", dict(j1=1.0), 5, W.log_mesh(1e-3, 100.0, 3)),                  # 31 pairs
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(BEYOND_20))
def test_rhs_beyond_20_pairs_every_element(name, precision):
    """Every element of one right-hand side on a seeded state against the
    oracle, in each launch form (one launch, three in turn, t beside s and u),
    which must also agree bitwise."""
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    lat, params, L, mesh = BEYOND_20[name]
    model = W.model(lat, **params)
    tables = build_tables(model, L)
    assert tables.n_pairs > 20
    ctx = Context(tables, mesh, precision=precision)
    orc = oracle.Oracle(model, L, mesh, threads=0)
    x = W.random_state(ctx.nf, ctx.ns, seed=_seed(name, precision), scale=0.3)
    lam = 0.29
    ref = orc.rhs(lam, expand_state(orc, tables, x))
    xs = torch.from_numpy(x).cuda()
    got = {}
    for form in ("one_launch", "separate", "concurrent"):
        _say(f"rhs beyond 20 pairs {name} ({ctx.ns} pairs) {precision} {form}")
        ctx.set_vertex_mode(form)
        got[form] = ctx.rhs(lam, xs).cpu().numpy()
        err = compare_vertex(orc, tables, ref, got[form])
        assert err <= (TOL if precision == "fp64" else 1e-5), (form, err)
    assert np.array_equal(got["one_launch"], got["separate"])
    assert np.array_equal(got["separate"], got["concurrent"])
    ctx.close()


@pytest.mark.parametrize("name", ["square_L2_N8", "honeycomb_L3_N6"])
def test_rhs_initial_state_and_init_kernel(name):
    torch, tables, ctx, orc = _setup(name)
    x = ctx.init_state()
    x0 = orc.initial_state()
    assert compare_vertex(orc, tables, x0, x.cpu().numpy()) == 0.0
    for lam in (0.05, 2.0):
        d = ctx.rhs(lam, x).cpu().numpy()
        assert compare_vertex(orc, tables, orc.rhs(lam, x0), d) <= 1e-13


@pytest.mark.parametrize("name", list(CASES))
def test_chi_and_structure_factor(name):
    torch, tables, ctx, orc = _setup(name)
    x = W.random_state(ctx.nf, ctx.ns, seed=3)
    xo = expand_state(orc, tables, x)
    for lam in (0.02, 0.7):
        _say(f"chi {name} lam={lam}")
        chi = ctx.chi(lam, torch.from_numpy(x).cuda()).cpu().numpy()
        zz, dd = orc.chi(lam, xo)
        assert compare_chi(orc, tables, zz, dd, chi) <= TOL
        kp = np.random.default_rng(1).uniform(-math.pi, math.pi, (37, 3))
        kp[:, 2] = 0.0 if name.startswith(("square", "honeycomb")) else kp[:, 2]
        ck = ctx.chi_k(torch.from_numpy(chi.reshape(-1)).cuda(), torch.from_numpy(kp).cuda()).cpu().numpy()
        ref = orc.chi_k(zz, kp)
        assert np.abs(ck - ref).max() <= TOL * np.abs(ref).max()


@pytest.mark.parametrize("name", ["honeycomb_L3_N6", "pyrochlore_L2_N5"])
def test_chi_sites_layout(name):
    """pffrg_chi_sites: chi in the observable-file layout (per basis site and
    site within range) equals the oracle's correlations of every (basis site,
    site), sites matched by position."""
    torch, tables, ctx, orc = _setup(name)
    x = W.random_state(ctx.nf, ctx.ns, seed=_seed(name, "sites"))
    xo = expand_state(orc, tables, x)
    chi = ctx.chi(0.3, torch.from_numpy(x).cuda())
    lay = ctx.chi_sites(chi).cpu().numpy()
    zz, dd = orc.chi(0.3, xo)
    err = compare_chi_sites(orc, tables, lay, np.stack([zz, dd]), chi.cpu().numpy())
    _say(f"chi sites {name}: {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("scheme", ["euler", "rk4"])
def test_single_steps(scheme):
    torch, tables, ctx, orc = _setup("honeycomb_L3_N6")
    x = W.random_state(ctx.nf, ctx.ns, seed=21, scale=0.1)
    xd = torch.from_numpy(x).cuda()
    xo = expand_state(orc, tables, x)
    l0, l1 = 0.9, 0.8
    ctx.step(scheme, l0, l1, xd)
    ref = orc.euler_step(l0, l1, xo) if scheme == "euler" else orc.rk4_step(l0, l1, xo)
    assert compare_vertex(orc, tables, ref, xd.cpu().numpy()) <= TOL


def test_rk4_flow_square_tiny_with_chi_every_step():
    """The small workload end to end: square L=2, 8 frequencies, 40 RK4 steps
    from Lambda=50 to 0.5, chi compared at every step."""
    torch, tables, ctx, orc = _setup("square_L2_N8")
    wl = W.workload("square_tiny")
    x = ctx.init_state()
    got = []
    ctx.flow(x, schedule=wl.schedule, scheme="rk4",
             observer=lambda lam, chi, ck: got.append((lam, chi.cpu().numpy().copy())) and 0)
    ref_chi = []
    xo = orc.flow(wl.schedule, observer=lambda lam, xs: ref_chi.append((lam, orc.chi(lam, xs))))
    assert compare_vertex(orc, tables, xo, x.cpu().numpy()) <= TOL
    assert len(got) == len(ref_chi) == len(wl.schedule) - 1
    for (lg, cg), (lr, (zz, dd)) in zip(got, ref_chi):
        assert lg == lr
        assert compare_chi(orc, tables, zz, dd, cg) <= TOL


@pytest.mark.parametrize("which", ["square_j1j2", "pyrochlore"])
def test_full_size_rhs_sampled(which):
    """The library at full workload size; the oracle computes every element of
    a sample of frequency triples (mesh corners, diagonal, random)."""
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    wl = W.workload(which)
    model = wl.model()
    tables = build_tables(model, wl.range)
    ctx = Context(tables, wl.mesh)
    orc = oracle.Oracle(model, wl.range, wl.mesh, threads=0)
    nf = ctx.nf
    x = W.random_state(nf, ctx.ns, seed=5, scale=0.2)
    lam = 0.21
    _say(f"full-size rhs {which} nf={nf} ns={ctx.ns}")
    d = ctx.rhs(lam, torch.from_numpy(x).cuda()).cpu().numpy()
    xo = expand_state(orc, tables, x)
    dsig = orc.sigma_rhs(lam, xo)
    assert np.abs(dsig - d[:nf]).max() <= TOL * np.abs(dsig).max()
    rng = np.random.default_rng(2)
    tri = [(0, 0, 0), (nf - 1, nf - 1, nf - 1), (nf - 1, 0, 0), (nf - 1, nf // 2, nf - 1)]
    for _ in range(4 if which == "pyrochlore" else 8):
        a = int(rng.integers(nf)); c = int(rng.integers(a + 1)); t = int(rng.integers(nf))
        tri.append((a, t, c))
    ref = orc.vertex_rhs_triples(lam, xo, dsig, tri)
    assert compare_triples(orc, tables, tri, ref, d) <= TOL


def test_adaptive_dopri_flow_matches_oracle():
    """Dormand-Prince 5(4) in ln Lambda with breakpoints at w_n/2: the accepted
    cutoffs and the final state agree with the oracle's controller."""
    torch, tables, ctx, orc = _setup("square_L2_N8")
    x = ctx.init_state()
    got = []
    n = ctx.flow(x, scheme="dopri54", lam_start=50.0, lam_stop=0.5, rtol=1e-5, atol=1e-8, h0=0.05,
                 hmin=1e-10, observer=lambda lam, chi, ck: got.append(lam) and 0)
    xo, lams = orc.dopri_flow(50.0, 0.5, 1e-5, 1e-8, 0.05, 1e-10)
    assert n == len(lams) == len(got)
    assert np.abs(np.array(got) - np.array(lams)).max() <= 1e-12 * 50
    assert compare_vertex(orc, tables, xo, x.cpu().numpy()) <= TOL


def test_flow_reports_divergence_and_keeps_last_finite_state():
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    from paper_2109_13317_amd._lib import PffrgError, EDIVERGED
    mesh = W.log_mesh(0.01, 10.0, 5)
    ctx = Context(build_tables(W.model("square", j1=1e200), 1), mesh)
    x = ctx.init_state()
    x0 = x.clone()
    with pytest.raises(PffrgError) as ei:
        ctx.flow(x, schedule=[5.0, 4.0, 3.0], scheme="rk4")
    assert ei.value.status == EDIVERGED
    assert torch.equal(x, x0)


@pytest.mark.parametrize("L,nf", [(0, 2), (0, 3), (1, 2)])
def test_degenerate_lattices_and_meshes(L, nf):
    """Range 0 (the on-site pair only, one lattice-sum term) and the smallest
    meshes (2 and 3 frequencies): right-hand side, chi and an RK4 step."""
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    model = W.model("square", j1=0.8, j2=0.3)
    mesh = W.log_mesh(0.05, 20.0, nf)
    tables = build_tables(model, L)
    ctx = Context(tables, mesh)
    orc = oracle.Oracle(model, L, mesh, threads=0)
    x = W.random_state(nf, ctx.ns, seed=31 + L + nf)
    xo = expand_state(orc, tables, x)
    for lam in (0.01, 0.5 * mesh[-1], 1.3, 40.0):
        _say(f"degenerate L={L} nf={nf} lam={lam}")
        d = ctx.rhs(lam, torch.from_numpy(x).cuda()).cpu().numpy()
        assert compare_vertex(orc, tables, orc.rhs(lam, xo), d) <= TOL
        chi = ctx.chi(lam, torch.from_numpy(x).cuda()).cpu().numpy()
        zz, dd = orc.chi(lam, xo)
        assert compare_chi(orc, tables, zz, dd, chi) <= TOL
    xd = torch.from_numpy(x).cuda()
    ctx.step("rk4", 2.0, 1.5, xd)
    assert compare_vertex(orc, tables, orc.rk4_step(2.0, 1.5, xo), xd.cpu().numpy()) <= TOL


def test_largest_mesh_sampled():
    """The largest supported mesh (128 frequencies, 1.06 M frequency triples)
    on a range-1 square lattice: the self-energy derivative in full and the
    vertex derivative on sampled triples (mesh ends, diagonal, random)."""
    import torch
    import oracle
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    model = W.model("square", j1=1.0)
    mesh = W.log_mesh(1e-3, 100.0, 128)
    tables = build_tables(model, 1)
    ctx = Context(tables, mesh)
    orc = oracle.Oracle(model, 1, mesh, threads=0)
    nf = ctx.nf
    x = W.random_state(nf, ctx.ns, seed=8, scale=0.2)
    lam = float(mesh[64]) * 0.5
    d = ctx.rhs(lam, torch.from_numpy(x).cuda()).cpu().numpy()
    xo = expand_state(orc, tables, x)
    dsig = orc.sigma_rhs(lam, xo)
    assert np.abs(dsig - d[:nf]).max() <= TOL * np.abs(dsig).max()
    rng = np.random.default_rng(4)
    tri = [(0, 0, 0), (nf - 1, nf - 1, nf - 1), (nf - 1, 0, 0), (64, 64, 64), (127, 3, 126)]
    for _ in range(6):
        a = int(rng.integers(nf)); c = int(rng.integers(a + 1)); t = int(rng.integers(nf))
        tri.append((a, t, c))
    ref = orc.vertex_rhs_triples(lam, xo, dsig, tri)
    assert compare_triples(orc, tables, tri, ref, d) <= TOL


@pytest.mark.parametrize("lat,params,L,nf,precision", [
    ("square", dict(j1=1.0), 2, 8, "fp64"),                      # 4 pairs
    ("honeycomb", dict(j1=0.6, j2=0.3, j3=0.45), 6, 10, "fp64"),  # 14 pairs
    ("square", dict(j1=1.0, j2=0.5), 7, 32, "fp64"),             # 20 pairs, the bench workload
    ("square", dict(j1=1.0, j2=0.5), 7, 32, "fp32"),
    ("pyrochlore", dict(j1=1.0), 5, 48, "fp64"),                 # 31 pairs, 3.5 M elements (past one grid)
])
def test_profiling_mask_times_only_the_named_kernels(lat, params, L, nf, precision):
    """Events recorded around the named launches only.  The default runs the
    three channels as one launch; timing a single channel runs them as three
    launches: the derivatives agree bitwise."""
    import torch
    from paper_2109_13317_amd import _lib, build_tables
    from paper_2109_13317_amd.flow import Context
    ctx = Context(build_tables(W.model(lat, **params), L), W.log_mesh(1e-3, 100.0, nf), precision=precision)
    _say(f"{lat} L={L} nf={nf} {precision}: {ctx.ns} pairs")
    x = torch.from_numpy(W.random_state(ctx.nf, ctx.ns, seed=3, scale=0.2)).cuda()
    ref = ctx.rhs(0.7, x).clone()
    ctx.set_profiling(True, kernels=("vertex_t",))
    out = ctx.rhs(0.7, x)
    out = ctx.rhs(0.7, x, out)
    ms_t, n_t = ctx.profile_read("vertex_t")
    assert n_t == 2 and ms_t > 0.0
    for k in ("sigma", "tables", "vertex", "vertex_s", "vertex_u", "vertex_stu"):
        assert ctx.profile_read(k) == (0.0, 0)
    assert torch.equal(out, ref)
    ctx.set_vertex_mode("one_launch")
    ctx.set_profiling(True, kernels=("vertex_stu",))
    out = ctx.rhs(0.7, x, out)
    ms, n = ctx.profile_read("vertex_stu")
    assert n == 1 and ms > 0.0 and ctx.profile_read("vertex_t") == (0.0, 0)
    ctx.set_profiling(False)
    assert torch.equal(out, ref)
    with pytest.raises(_lib.PffrgError):           # a bit past the last kernel id
        _lib.check(ctx.lib.pffrg_set_profiling_mask(ctx.handle, 1 << 7))


@pytest.mark.parametrize("lat,params,L,nf,precision", [
    ("square", dict(j1=1.0), 2, 8, "fp64"),                      # 4 pairs
    ("honeycomb", dict(j1=0.6, j2=0.3, j3=0.45), 6, 10, "fp32"),  # 14 pairs
    ("square", dict(j1=1.0, j2=0.5), 7, 32, "fp64"),             # 20 pairs
    ("pyrochlore", dict(j1=1.0), 5, 48, "fp64"),                 # 31 pairs
    ("pyrochlore", dict(j1=1.0), 5, 48, "fp32"),
])
def test_vertex_launch_modes_agree_bitwise(lat, params, L, nf, precision):
    """One launch, three launches in turn, and s+u beside a concurrent t
    launch on the context's second stream: the same sums in the same order,
    so the same bits, also when right-hand sides follow each other on the
    stream (the join must order the next stage after the t launch)."""
    import torch
    from paper_2109_13317_amd import _lib, build_tables
    from paper_2109_13317_amd.flow import Context
    ctx = Context(build_tables(W.model(lat, **params), L), W.log_mesh(1e-3, 100.0, nf), precision=precision)
    _say(f"launch modes {lat} L={L} nf={nf} {precision}: {ctx.ns} pairs")
    x = torch.from_numpy(W.random_state(ctx.nf, ctx.ns, seed=4, scale=0.2)).cuda()
    res = {}
    for mode in ("one_launch", "separate", "concurrent", "auto"):
        ctx.set_vertex_mode(mode)
        y = x.clone()
        ctx.step("rk4", 0.7, 0.6, y)                # four right-hand sides back to back
        d = ctx.rhs(0.45, y)
        torch.cuda.synchronize()
        res[mode] = (y.clone(), d.clone())
    for mode in ("separate", "concurrent", "auto"):
        assert torch.equal(res[mode][0], res["one_launch"][0]), mode
        assert torch.equal(res[mode][1], res["one_launch"][1]), mode
    with pytest.raises(_lib.PffrgError):
        _lib.check(ctx.lib.pffrg_set_vertex_mode(ctx.handle, 3))


def test_measure_peaks_is_plausible():
    """The on-device peak measurement returns finite rates in a plausible
    range (it feeds the roofline fractions of the benchmark)."""
    from paper_2109_13317_amd.flow import measure_peaks
    pk = measure_peaks()
    _say(f"measured peaks {pk}")
    assert 1.0 < pk["fp64_fma_tflops"] < 200.0
    assert 1.0 < pk["fp32_fma_tflops"] < 400.0
    assert 100.0 < pk["hbm_copy_gbs"] < 20000.0
    for k in ("l1_load_tbs", "l1_load_2row_tbs", "lds_read_tbs"):
        assert 1.0 < pk[k] < 1000.0, k
