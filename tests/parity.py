"""Helpers that put the library's reduced flow state next to the oracle's.

The oracle keeps the vertex for every (basis site b, site k within range of
b) separately; the library keeps one value per symmetry-reduced pair.  Sites
are matched by their Cartesian positions, so the comparison trusts neither
side's site numbering.
"""

from __future__ import annotations

import numpy as np


def pair_map(orc, tables) -> np.ndarray:
    """pmap[b, k] = reduced pair of the oracle's site k of basis b (-1 pad)."""
    lat = orc.lat
    pmap = np.full((lat.nb, lat.ns), -1, dtype=np.int64)
    for b in range(lat.nb):
        prod = {tuple(np.round(tables.site_pos[b, k], 6)): int(tables.site_pair[b, k])
                for k in range(tables.n_sites_total) if tables.site_pair[b, k] >= 0}
        for k in range(lat.nsites[b]):
            key = tuple(np.round(lat.site_pos[b, k], 6))
            pmap[b, k] = prod[key]
    return pmap


def _reduced_views(x, nf, ns):
    n_su = nf * (nf + 1) // 2
    v = n_su * nf * ns
    return x[:nf], x[nf:nf + v].reshape(n_su, nf, ns), x[nf + v:nf + 2 * v].reshape(n_su, nf, ns)


def expand_state(orc, tables, x_red: np.ndarray) -> np.ndarray:
    """Oracle-layout state holding the same values as a reduced state."""
    pmap = pair_map(orc, tables)
    nf, ns = orc.nf, tables.n_pairs
    sig, gs, gd = _reduced_views(np.asarray(x_red), nf, ns)
    out = orc.initial_state() * 0.0
    osig, ogs, ogd = orc.split(out)
    osig[:] = sig
    for b in range(orc.lat.nb):
        n = orc.lat.nsites[b]
        ogs[b, :, :, :n] = gs[:, :, pmap[b, :n]]
        ogd[b, :, :, :n] = gd[:, :, pmap[b, :n]]
    return out


def compare_vertex(orc, tables, ref: np.ndarray, red: np.ndarray) -> float:
    """max |oracle - library| / max |oracle| over sigma and every vertex
    element of every (basis, site) of the oracle."""
    pmap = pair_map(orc, tables)
    nf, ns = orc.nf, tables.n_pairs
    sig, gs, gd = _reduced_views(np.asarray(red), nf, ns)
    rsig, rgs, rgd = orc.split(ref)
    err = np.abs(rsig - sig).max()
    scale = max(np.abs(rsig).max(), np.abs(rgs).max(), np.abs(rgd).max(), 1e-300)
    for b in range(orc.lat.nb):
        n = orc.lat.nsites[b]
        err = max(err, np.abs(rgs[b, :, :, :n] - gs[:, :, pmap[b, :n]]).max(),
                  np.abs(rgd[b, :, :, :n] - gd[:, :, pmap[b, :n]]).max())
    return float(err / scale)


def compare_triples(orc, tables, triples, ref_tr: np.ndarray, red: np.ndarray) -> float:
    """Like compare_vertex for the oracle's per-triple output [nq, nb, ns, 2]."""
    pmap = pair_map(orc, tables)
    nf, ns = orc.nf, tables.n_pairs
    _, gs, gd = _reduced_views(np.asarray(red), nf, ns)
    err, scale = 0.0, 1e-300
    for q, (a, t, c) in enumerate(triples):
        su = a * (a + 1) // 2 + c
        for b in range(orc.lat.nb):
            n = orc.lat.nsites[b]
            r = ref_tr[q, b, :n]
            err = max(err, np.abs(r[:, 0] - gs[su, t, pmap[b, :n]]).max(),
                      np.abs(r[:, 1] - gd[su, t, pmap[b, :n]]).max())
            scale = max(scale, np.abs(r).max())
    return float(err / scale)


def compare_chi(orc, tables, zz, dd, chi_red: np.ndarray) -> float:
    pmap = pair_map(orc, tables)
    chi_red = np.asarray(chi_red).reshape(2, -1)
    err, scale = 0.0, 1e-300
    for b in range(orc.lat.nb):
        n = orc.lat.nsites[b]
        err = max(err, np.abs(zz[b, :n] - chi_red[0, pmap[b, :n]]).max(),
                  np.abs(dd[b, :n] - chi_red[1, pmap[b, :n]]).max())
        scale = max(scale, np.abs(zz[b, :n]).max(), np.abs(dd[b, :n]).max())
    return float(err / scale)


def compare_parts(orc, tables, ref: np.ndarray, red: np.ndarray) -> tuple[float, float]:
    """(sigma error / max |sigma|, vertex error / max |vertex|): the two parts
    of a state or derivative measured on their own scales."""
    pmap = pair_map(orc, tables)
    nf, ns = orc.nf, tables.n_pairs
    sig, gs, gd = _reduced_views(np.asarray(red), nf, ns)
    rsig, rgs, rgd = orc.split(ref)
    es = np.abs(rsig - sig).max() / max(np.abs(rsig).max(), 1e-300)
    ev, scale = 0.0, max(np.abs(rgs).max(), np.abs(rgd).max(), 1e-300)
    for b in range(orc.lat.nb):
        n = orc.lat.nsites[b]
        ev = max(ev, np.abs(rgs[b, :, :, :n] - gs[:, :, pmap[b, :n]]).max(),
                 np.abs(rgd[b, :, :, :n] - gd[:, :, pmap[b, :n]]).max())
    return float(es), float(ev / scale)


def restrict_state(orc, tables, x_unred: np.ndarray) -> np.ndarray:
    """Reduced-layout state holding, for every reduced pair, the values of
    one of its unreduced copies (the first (basis, site) mapped to it).  For
    a symmetric state this inverts expand_state."""
    pmap = pair_map(orc, tables)
    nf, ns = orc.nf, tables.n_pairs
    rep = {}
    for b in range(orc.lat.nb):
        for k in range(orc.lat.nsites[b]):
            rep.setdefault(int(pmap[b, k]), (b, k))
    assert len(rep) == ns
    sig, gs, gd = orc.split(np.asarray(x_unred))
    n_su = nf * (nf + 1) // 2
    out = np.zeros(nf + 2 * n_su * nf * ns)
    osig, ogs, ogd = _reduced_views(out, nf, ns)
    osig[:] = sig
    for p, (b, k) in rep.items():
        ogs[:, :, p] = gs[b, :, :, k]
        ogd[:, :, p] = gd[b, :, :, k]
    return out
