"""The split of the tabulated lattice-sum terms into lane runs (term_runs in
csrc/kernels_flow.h), compiled for the host: for the pair term counts of the
workloads and for random and edge-case lists, the runs cover every term of
every pair exactly once, in order, each within one pair; the run offsets
agree with the runs; at most 64 runs and the rest empty; and the longest run
is as short as any split with at most 64 runs within pairs allows (the
smallest S with sum_p ceil(n_p / S) <= 64, found here by direct search).
Host code only (no GPU)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WAVE = 64


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not found")


@pytest.fixture(scope="module")
def split(tmp_path_factory):
    exe = tmp_path_factory.mktemp("runs") / "term_runs_dump"
    src = os.path.join(ROOT, "tests", "term_runs_dump.cpp")
    subprocess.run([_hipcc(), "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2109_13317_amd", "csrc"), src, "-o", str(exe)],
                   check=True, capture_output=True, text=True, timeout=300)

    def run(cases):
        text = "\n".join(" ".join(map(str, [len(o) - 1, *o])) for o in cases) + "\n"
        out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, timeout=60, check=True).stdout
        res, cur = [], None
        for line in out.splitlines():
            f = line.split()
            if f[0] == "N":
                cur = {"n": int(f[1]), "runs": [], "off": []}
                res.append(cur)
            elif f[0] == "R":
                cur["runs"].append((int(f[2]), int(f[3])))
            else:
                cur["off"].append(int(f[2]))
        return res
    return run


def _best_max(lens):
    """Smallest S with sum ceil(n / S) <= 64 over the non-empty lists."""
    lens = [n for n in lens if n > 0]
    if not lens:
        return 0
    for S in range(1, max(lens) + 1):
        if sum(-(-n // S) for n in lens) <= WAVE:
            return S
    raise AssertionError("more than 64 non-empty pairs")


def _check(off, r):
    ns = len(off) - 1
    lens = np.diff(off)
    n = r["n"]
    assert 0 <= n <= WAVE
    assert r["off"][0] == 0 and r["off"][ns] == n
    for x, y in r["runs"][n:]:
        assert x == y == 0
    for p in range(ns):
        a, b = r["off"][p], r["off"][p + 1]
        assert a <= b
        runs = r["runs"][a:b]
        if lens[p] == 0:
            assert not runs
            continue
        # consecutive, non-empty, inside pair p, covering it
        assert runs[0][0] == off[p] and runs[-1][1] == off[p + 1]
        for (x0, y0), (x1, y1) in zip(runs, runs[1:]):
            assert y0 == x1
        for x, y in runs:
            assert off[p] <= x < y <= off[p + 1]
        # near-equal lengths within the pair
        ls = [y - x for x, y in runs]
        assert max(ls) - min(ls) <= 1
    longest = max((y - x for x, y in r["runs"][:n]), default=0)
    assert longest == _best_max(lens), (longest, _best_max(lens))


def test_workload_term_lists(split):
    import workloads as W
    from paper_2109_13317_amd import build_tables
    offs = []
    for name in W.WORKLOAD_NAMES:
        wl = W.workload(name)
        offs.append([int(v) for v in build_tables(wl.model(), wl.range).rpa_off])
    res = split(offs)
    for off, r in zip(offs, res):
        _check(off, r)
    pyro = res[W.WORKLOAD_NAMES.index("pyrochlore")]
    # pyrochlore range 5: 31 pairs, 3007 terms, the longest pair 188; split
    # into 64 runs of at most 61 terms
    assert pyro["n"] == 64
    assert max(y - x for x, y in pyro["runs"]) == 61


def test_random_and_edge_lists(split):
    rng = np.random.default_rng(7)
    offs = [[0, 0], [0, 1], [0, 0, 0, 5], [0, 64], [0, 1000], list(range(0, 65)), [0] * 33,
            list(np.cumsum([0] + [1] * 64)), [0, 3, 3, 3, 200, 201]]
    for _ in range(60):
        ns = int(rng.integers(1, WAVE + 1))
        lens = rng.integers(0, 300, ns) * (rng.random(ns) < 0.9)
        offs.append([0] + [int(v) for v in np.cumsum(lens)])
    for off, r in zip(offs, split(offs)):
        _check(off, r)
