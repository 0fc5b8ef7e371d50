"""Host-side checks that need no GPU: the C ABI's exports and argument
validation, and the symmetry-reduced lattice tables of the front end."""

import ctypes
import dataclasses
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2109_13317_amd.lattice import build_tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "pffrg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pffrg_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2109_13317_amd import _lib
    lib = _lib.load()
    names = _declared_symbols()
    assert "pffrg_rhs" in names and "pffrg_create" in names
    for n in names:
        assert hasattr(lib, n), n


def test_create_rejects_bad_inputs_before_touching_the_gpu():
    from paper_2109_13317_amd import _lib
    lib = _lib.load()
    t = build_tables(W.model("square", j1=1.0), 1)
    arrs = [np.ascontiguousarray(a) for a in (t.swap, t.mult, t.rpa_off, t.rpa_ka, t.rpa_kb, t.rpa_cnt)]
    arrs += [t.coupling.astype(np.float64), t.site_pair.astype(np.int32), t.site_pos, t.basis_pos]
    p = [ctypes.c_void_p(a.ctypes.data) for a in arrs]
    lat = _lib.Lattice(t.n_pairs, *p[:7], t.n_basis, t.n_sites_total, *p[7:])
    h = ctypes.c_void_p()
    for mesh in ([1.0], [0.5, 0.4], [0.0, 1.0], [1.0, float("nan")]):
        m = np.array(mesh)
        msh = _lib.Mesh(len(m), ctypes.c_void_p(m.ctypes.data))
        st = lib.pffrg_create(ctypes.byref(lat), ctypes.byref(msh), _lib.FP64, None, ctypes.byref(h))
        assert st == _lib.EINVAL and not h.value
        assert lib.pffrg_last_error()
    bad = arrs[0].copy(); bad[0] = 1
    lat2 = _lib.Lattice(t.n_pairs, ctypes.c_void_p(bad.ctypes.data), *p[1:7], t.n_basis, t.n_sites_total, *p[7:])
    m = np.array([0.1, 1.0])
    msh = _lib.Mesh(2, ctypes.c_void_p(m.ctypes.data))
    assert lib.pffrg_create(ctypes.byref(lat2), ctypes.byref(msh), _lib.FP64, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.pffrg_create(None, ctypes.byref(msh), _lib.FP64, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.pffrg_rhs(None, 1.0, None, None) == _lib.EINVAL
    assert lib.pffrg_status_string(_lib.EDIVERGED) == b"PFFRG_EDIVERGED"


def test_create_rejects_each_malformed_table():
    """One field of valid tables corrupted at a time: pffrg_create returns
    the documented status with a message naming the field, leaves the handle
    NULL, and does so before any HIP call (this runs without a GPU)."""
    from paper_2109_13317_amd import _lib
    from paper_2109_13317_amd.flow import _lattice_struct
    lib = _lib.load()
    t = build_tables(W.model("square", j1=1.0, j2=0.5), 2)
    ns = t.n_pairs
    mesh = np.array([0.1, 1.0, 10.0])
    cases = [
        ("swap", 1, ns, "swap out of range"), ("swap", 1, -1, "swap out of range"),
        ("mult", 1, 0, "mult"), ("rpa_off", 0, 1, "bad rpa_off"),
        ("rpa_off", 1, int(t.rpa_off[2]) + 1, "rpa_off not ascending"),
        ("rpa_ka", 0, ns, "rpa term pair"), ("rpa_kb", 0, -1, "rpa term pair"),
        ("rpa_cnt", 0, 0, "rpa_cnt"), ("rpa_cnt", 0, 32768, "rpa_cnt"),
        ("coupling", 1, float("nan"), "couplings must be finite"),
        ("coupling", 1, float("inf"), "couplings must be finite"),
        ("site_pair", (0, 0), ns, "site_pair"), ("site_pair", (0, 1), -2, "site_pair"),
    ]
    h = ctypes.c_void_p()
    msh = _lib.Mesh(3, ctypes.c_void_p(mesh.ctypes.data))

    def create(tab, m=msh, prec=_lib.FP64):
        lat, keep = _lattice_struct(tab)
        st = lib.pffrg_create(ctypes.byref(lat), ctypes.byref(m), prec, None, ctypes.byref(h))
        assert not h.value
        return st, lib.pffrg_last_error().decode()

    for field, idx, val, msg in cases:
        a = np.array(getattr(t, field), copy=True)
        a[idx] = val
        st, err = create(dataclasses.replace(t, **{field: a}))
        assert st == _lib.EINVAL and msg in err, (field, val, err)
    assert create(t, prec=7) == (_lib.EINVAL, "unknown precision")
    st, err = create(dataclasses.replace(t, n_pairs=33))
    assert st == _lib.EUNSUPPORTED and "32" in err
    st, err = create(dataclasses.replace(t, n_pairs=0))
    assert st == _lib.EINVAL and "incomplete" in err
    st, err = create(dataclasses.replace(t, n_basis=0))
    assert st == _lib.EINVAL and "site map" in err
    big = np.geomspace(0.01, 50.0, 129)
    st, err = create(t, m=_lib.Mesh(129, ctypes.c_void_p(big.ctypes.data)))
    assert st == _lib.EUNSUPPORTED and "128" in err
    lat, keep = _lattice_struct(t)
    assert lib.pffrg_create(ctypes.byref(lat), ctypes.byref(msh), _lib.FP64, None, None) == _lib.EINVAL


# ---------------------------------------------------------- lattice tables -

def test_reduced_pair_counts():
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "lattice_counts.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        t = build_tables(W.model(r[0], j1=1.0), int(r[1]))
        assert t.n_sites_total == int(r[2])
        if r[3] != "-":
            assert t.n_pairs == int(r[3])


@pytest.mark.parametrize("lattice,L,ns,order", [("square", 7, 20, 16), ("square", 2, 4, 16),
                                                ("honeycomb", 6, 14, 12), ("pyrochlore", 5, 31, 12),
                                                ("cubic", 4, 11, 48)])
def test_reduction_structure(lattice, L, ns, order):
    """Orbit counts of the point group fixing the reference site: square D4
    (x z-mirror), honeycomb D3 (x z-mirror), pyrochlore D3d, cubic Oh."""
    t = build_tables(W.model(lattice, j1=1.0), L)
    assert t.n_pairs == ns and t.stabiliser_order == order
    assert t.mult.sum() == t.n_sites_total
    assert np.all(t.swap[t.swap] == np.arange(ns))          # exchange is an involution
    assert t.swap[0] == 0 and t.mult[0] == 1
    # every site of every basis row maps to a pair, each pair hit mult times per row
    for b in range(t.n_basis):
        row = t.site_pair[b][t.site_pair[b] >= 0]
        assert np.array_equal(np.bincount(row, minlength=ns), t.mult)


@pytest.mark.parametrize("lattice,params,L", [("square", dict(j1=1.0, j2=0.5), 4),
                                              ("honeycomb", dict(j1=0.7, j2=0.3, j3=0.4), 4),
                                              ("pyrochlore", dict(j1=1.0), 3)])
def test_lattice_sum_tables_against_brute_force(lattice, params, L):
    """sum_{(ka,kb)} cnt g_ka g_kb == sum over lattice sites j of
    J(i_ref, j) J(j, j_p) with both distances within range, by brute force
    over positions, for an arbitrary pair-dependent test field g."""
    m = W.model(lattice, **params)
    t = build_tables(m, L)
    rng = np.random.default_rng(0)
    g = rng.normal(size=t.n_pairs)
    cell = W.unit_cell(lattice)
    # brute force: enumerate sites, bond distance by BFS on positions
    pos = {}
    reach = L + 2
    for d0 in range(-2 * reach, 2 * reach + 1):
        for d1 in range(-2 * reach, 2 * reach + 1):
            for d2 in (range(-2 * reach, 2 * reach + 1) if lattice == "pyrochlore" else (0,)):
                for b in range(cell.n_basis):
                    pos[(d0, d1, d2, b)] = cell.position((d0, d1, d2), b)
    keys = list(pos)
    P = np.array([pos[k] for k in keys])
    bond_len = min(np.linalg.norm(cell.position(bd[2:], bd[1]) - cell.basis[bd[0]]) for bd in cell.bonds)

    def bfs(src):
        from collections import deque
        dist = {src: 0}
        q = deque([src])
        while q:
            k = q.popleft()
            if dist[k] == L:
                continue
            dd = np.linalg.norm(P - pos[k], axis=1)
            for j in np.nonzero(np.abs(dd - bond_len) < 1e-6)[0]:
                kk = keys[j]
                if kk not in dist:
                    dist[kk] = dist[k] + 1
                    q.append(kk)
        return dist

    ref_site = (0, 0, 0, 0)
    d0 = bfs(ref_site)
    pair_of = {}
    for k in range(t.n_sites_total):
        if t.site_pair[0, k] >= 0:
            pair_of[tuple(np.round(t.site_pos[0, k], 6))] = int(t.site_pair[0, k])

    def pair(i, j):
        """reduced pair of (i, j) by translating i to the reference cell; only
        needed for i on basis 0 or for the field value through positions."""
        return pair_of.get(tuple(np.round(pos[j] - pos[i] + pos[ref_site], 6)))

    for p in range(t.n_pairs):
        rep = next(k for k in d0 if pair(ref_site, k) == p)
        dp = bfs(rep)
        table = sum(int(t.rpa_cnt[q]) * g[t.rpa_ka[q]] * g[t.rpa_kb[q]]
                    for q in range(t.rpa_off[p], t.rpa_off[p + 1]))
        if cell.n_basis == 1:
            brute = sum(g[pair(ref_site, j)] * g[pair(j, rep)] for j in d0 if j in dp)
            assert abs(table - brute) < 1e-9, (p, table, brute)
        # term count: sites within range of both ends
        n_terms = int(t.rpa_cnt[t.rpa_off[p]:t.rpa_off[p + 1]].sum())
        assert n_terms == sum(1 for j in d0 if j in dp), p


def test_batch_create_rejects_bad_inputs_before_touching_the_gpu():
    from paper_2109_13317_amd import _lib
    from paper_2109_13317_amd.flow import _lattice_struct
    lib = _lib.load()
    small = build_tables(W.model("square", j1=1.0), 1)
    big = build_tables(W.model("pyrochlore", j1=1.0), 5)          # 31 pairs
    m = np.array([0.1, 1.0, 10.0])
    msh = _lib.Mesh(3, ctypes.c_void_p(m.ctypes.data))
    h = ctypes.c_void_p()
    lat_s, keep_s = _lattice_struct(small)
    lat_b, keep_b = _lattice_struct(big)
    arr = (ctypes.POINTER(_lib.Lattice) * 2)(ctypes.pointer(lat_s), ctypes.pointer(lat_b))
    assert lib.pffrg_batch_create(2, arr, ctypes.byref(msh), _lib.FP32, None, ctypes.byref(h)) == _lib.EUNSUPPORTED
    assert b"point 1" in lib.pffrg_last_error() and not h.value
    assert lib.pffrg_batch_create(0, arr, ctypes.byref(msh), _lib.FP32, None, ctypes.byref(h)) == _lib.EINVAL
    bad = np.array([1.0, 0.5])
    msh2 = _lib.Mesh(2, ctypes.c_void_p(bad.ctypes.data))
    assert lib.pffrg_batch_create(1, arr, ctypes.byref(msh2), _lib.FP64, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.pffrg_batch_create(1, arr, ctypes.byref(msh), 7, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.pffrg_batch_rhs(None, 1.0, None, None) == _lib.EINVAL


def test_chi_noalloc_rejects_bad_arguments_before_any_hip_call():
    """Argument checks of the no-allocation entry point run on the host before
    the device is touched (the fake device pointers are never dereferenced)."""
    from paper_2109_13317_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(256)
    cases = [((2, None, 1, fake, 0.5, fake, fake, None), _lib.EINVAL),
             ((2, fake, 1, fake, 0.5, fake, None, None), _lib.EINVAL),
             ((1, fake, 1, fake, 0.5, fake, fake, None), _lib.EINVAL),
             ((4, fake, 0, fake, 0.5, fake, fake, None), _lib.EINVAL),
             ((4, fake, 2, fake, 0.0, fake, fake, None), _lib.EINVAL),
             ((4, fake, 2, fake, float("inf"), fake, fake, None), _lib.EINVAL),
             ((129, fake, 2, fake, 0.5, fake, fake, None), _lib.EUNSUPPORTED),
             ((8, fake, 33, fake, 0.5, fake, fake, None), _lib.EUNSUPPORTED)]
    for args, want in cases:
        assert lib.pffrg_chi_noalloc(*args) == want, args
        assert lib.pffrg_last_error()
