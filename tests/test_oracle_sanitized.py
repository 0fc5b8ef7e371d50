"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is built a second time with gcc's address and undefined-behaviour
checks (-O1, every check fatal) and run in a child process (the sanitizer
runtime must be loaded first) on small lattices with and without pair
exchange: the right-hand side on several threads, the self-energy flow alone,
single elements and triples, and the correlations.  Its results must equal
the regular build's bit for bit: both builds keep IEEE FP64 semantics (no
contraction, no reassociation), so neither the optimisation level nor the
checks may change a result.
"""

import os
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r"""
import sys
import numpy as np
import oracle
import workloads as W

out = {}
for name, lat, params, L, nf in (("sq", "square", dict(j1=1.0, j2=0.4), 2, 5),
                                  ("hc", "honeycomb", dict(j1=1.0, j2=0.3, j3=0.2), 3, 4),
                                  ("py", "pyrochlore", dict(j1=1.0), 1, 3)):
    o = oracle.Oracle(W.model(lat, **params), L, W.log_mesh(0.02, 20.0, nf), threads=3)
    rng = np.random.default_rng(17)
    x = o.initial_state() + 0.2 * rng.normal(size=o.size)
    x[: o.nf] = -np.abs(x[: o.nf])
    for lam in (0.5 * float(o.mesh[1]), 0.3, 40.0):
        out[f"{name}_rhs_{lam}"] = o.rhs(lam, x)
        ds = o.sigma_rhs(lam, x)
        out[f"{name}_sig_{lam}"] = ds
        out[f"{name}_tri_{lam}"] = o.vertex_rhs_triples(lam, x, ds, [(o.nf - 1, 0, 0), (1, o.nf - 1, 1)])
        out[f"{name}_el_{lam}"] = o.vertex_rhs_element(lam, x, ds, o.lat.nb - 1, 1, o.nf - 1, 1, 0)
        zz, dd = o.chi(lam, x)
        out[f"{name}_chi_{lam}"] = np.concatenate([zz.ravel(), dd.ravel()])
np.savez(sys.argv[1], **out)
"""


def _run(tmp_path, lib, env_extra, tag):
    env = dict(os.environ, PYTHONPATH=ROOT, OMP_NUM_THREADS="3", **env_extra)
    if lib is not None:
        env["PFFRG_ORACLE_LIB"] = lib
    out = str(tmp_path / f"{tag}.npz")
    r = subprocess.run([sys.executable, "-c", CHILD, out], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return np.load(out)


def test_oracle_clean_under_address_and_ub_sanitizers(oracle_lib, tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not (os.path.isabs(asan) and os.path.exists(asan) and os.path.isabs(ubsan) and os.path.exists(ubsan)):
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = oracle_lib.build(force=True, out=str(tmp_path / "liborc_san.so"),
                           extra=("-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                                  "-fno-sanitize-recover=all"))
    san = _run(tmp_path, lib, {"LD_PRELOAD": f"{asan}:{ubsan}",
                                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}, "san")
    ref = _run(tmp_path, None, {}, "ref")
    assert set(san.files) == set(ref.files)
    for k in ref.files:
        assert np.array_equal(san[k], ref[k]), k
