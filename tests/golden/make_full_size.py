"""Write the oracle's results for the full-size parity cases (run on a CPU).

    python tests/golden/make_full_size.py [case ...]

Cases (workload sizes of the benchmark, seeded random states):
  square_j1j2_rk4     square J1-J2 (J2/J1 = 0.5), range 7, 32 log frequencies
                      1e-3..100: one classical RK4 step Lambda 0.6 -> 0.55
                      (four right-hand sides) of a random state;
  honeycomb_j123_rk4  honeycomb J1-J2-J3, range 6, 32 frequencies: one RK4
                      step Lambda 0.9 -> 0.8;
  pyrochlore_rhs      pyrochlore, range 5, 48 frequencies: the self-energy
                      flow and the vertex flow of 288 frequency triples (six
                      in every t row) at Lambda = 0.37.

Every stored value is computed by the FP64 oracle (``oracle/``) alone.  The
input is the seeded reduced random state of ``workloads.random_state``,
spread onto the oracle's unreduced lattice by site position (the mapping of
``tests/parity.py``, built from the host-side lattice tables; no GPU code is
loaded).  Each file records that pair map, so a test can refuse a file whose
pair numbering no longer matches the tables.  The oracle's result must
itself be constant on every orbit of reduced pairs (checked here to 1e-12),
which is what lets a reduced state be compared with it element by element.
The vertex values are a seeded sample of the elements (plus the self-energy
in full), with the largest magnitude of the whole result as the scale.
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from paper_2109_13317_amd.lattice import build_tables  # noqa: E402  (host tables only)
from tests.parity import expand_state, pair_map, restrict_state  # noqa: E402

N_SAMPLE = 20000

CASES = {
    "square_j1j2_rk4": dict(workload="square_j1j2", seed=11, scale=0.1, kind="rk4", lam=(0.6, 0.55)),
    "honeycomb_j123_rk4": dict(workload="honeycomb_j123", seed=12, scale=0.1, kind="rk4", lam=(0.9, 0.8)),
    "pyrochlore_rhs": dict(workload="pyrochlore", seed=13, scale=0.1, kind="rhs", lam=(0.37,)),
}


def _orbit_spread(orc, tables, y):
    """Largest difference between an unreduced element and its orbit's
    representative, relative to max |y|."""
    back = expand_state(orc, tables, restrict_state(orc, tables, y))
    return float(np.abs(back - y).max() / np.abs(y).max())


def make(name: str) -> str:
    c = CASES[name]
    wl = W.workload(c["workload"])
    model = wl.model()
    tables = build_tables(model, wl.range)
    orc = oracle.Oracle(model, wl.range, wl.mesh, threads=os.cpu_count() or 1)
    nf, ns = len(wl.mesh), tables.n_pairs
    x = W.random_state(nf, ns, seed=c["seed"], scale=c["scale"])
    xo = expand_state(orc, tables, x)
    rec = dict(workload=c["workload"], seed=c["seed"], scale=c["scale"], kind=c["kind"],
               lam=np.array(c["lam"]), nf=nf, ns=ns, pmap=pair_map(orc, tables),
               mesh=np.asarray(wl.mesh))
    t0 = time.perf_counter()
    if c["kind"] == "rk4":
        y = orc.rk4_step(c["lam"][0], c["lam"][1], xo)
        spread = _orbit_spread(orc, tables, y)
        assert spread <= 1e-12, spread
        yr = restrict_state(orc, tables, y)
        rng = np.random.default_rng(c["seed"] + 1000)
        idx = np.sort(rng.choice(np.arange(nf, yr.size), size=N_SAMPLE, replace=False))
        rec.update(sigma=yr[:nf], index=idx.astype(np.int64), value=yr[idx],
                   scale_max=float(np.abs(y).max()), orbit_spread=spread)
    else:
        lam = c["lam"][0]
        dsig = orc.sigma_rhs(lam, xo)
        rng = np.random.default_rng(c["seed"] + 1000)
        tri = []
        for t in range(nf):
            tri.append((nf - 1, t, 0))
            tri.append((t, t, t))
            for _ in range(4):
                a = int(rng.integers(nf))
                tri.append((a, t, int(rng.integers(a + 1))))
        tri = np.array(tri, dtype=np.int64)
        ref = orc.vertex_rhs_triples(lam, xo, dsig, tri)          # [nq, nb, ns_unred, 2]
        pm = rec["pmap"]
        red = np.zeros((len(tri), ns, 2))
        spread = 0.0
        for p in range(ns):
            bs, ks = np.nonzero(pm == p)
            v = ref[:, bs, ks, :]                                  # every copy of pair p
            red[:, p, :] = v[:, 0, :]
            spread = max(spread, float(np.abs(v - v[:, :1, :]).max()))
        spread /= float(np.abs(ref).max())
        assert spread <= 1e-12, spread
        rec.update(sigma=dsig, triples=tri, value=red, scale_max=float(np.abs(ref).max()),
                   orbit_spread=spread)
    rec["oracle_seconds"] = time.perf_counter() - t0
    out = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(out, **rec)
    print(f"{name}: {rec['oracle_seconds']:.1f} s, orbit spread {spread:.2e} -> {out}", flush=True)
    return out


if __name__ == "__main__":
    oracle.build(force=False)
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
