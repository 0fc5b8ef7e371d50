"""The compile-time tables of the TRI vertex kernels (csrc/kernels_tri.h),
compiled for the host, against the definition: for random vertices in the
real representation (Gamma = r where xi(mu) xi(nu) = 1, i r where it is -1,
Eq. 18) every channel product of Eq. 24, formed literally from 2x2x2x2 spin
tensors (Eq. 25) with the spin sums in the leg order the paper prints and
projected back with Pauli traces, equals what the table's terms give; the
parts the real representation drops vanish; and the correlation exchange
coefficients equal the spin-index sum of Eq. 30 with legs 1' and 2'
exchanged.  Host code only (no GPU)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIG = np.array([[[1, 0], [0, 1]], [[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=complex)
XI = np.array([1.0, -1.0, -1.0, -1.0])
XIXI = np.outer(XI, XI)
# the spin sums of Eq. 24 per product, in the legs of the two vertices
# (s: (1'2';34)(34;12); u: (42';13)(1'3;42); t: RPA (1'4;13)(32';42) with the
# leading minus, corrections (1'4;13)(2'3;42) and (41';13)(32';42))
FORMS = {0: ("pqcd,cdab->pqab", 1.0), 1: ("dqac,pcdb->pqab", 1.0), 2: ("pdac,qcdb->pqab", 1.0),
         3: ("dpac,cqdb->pqab", 1.0), 4: ("pdac,cqdb->pqab", -1.0)}


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not found")


@pytest.fixture(scope="module")
def tables(tmp_path_factory):
    exe = tmp_path_factory.mktemp("tri") / "tri_tables_dump"
    src = os.path.join(ROOT, "tests", "tri_tables_dump.cpp")
    subprocess.run([_hipcc(), "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2109_13317_amd", "csrc"), src, "-o", str(exe)],
                   check=True, capture_output=True, text=True, timeout=300)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60, check=True).stdout
    terms = {ch: [] for ch in range(5)}
    chi_x = np.zeros((16, 16))
    for line in out.splitlines():
        f = line.split()
        if f[0] == "T":
            ch, i, c1, c2, q, k = map(int, f[1:])
            terms[ch].append((c1, c2, q, k))
        else:
            chi_x[int(f[1]), int(f[2])] = int(f[3])
    return terms, chi_x


def _tensor(G):
    return np.einsum("mn,mpa,nqb->pqab", G, SIG, SIG)


def _basis(P):
    return 0.25 * np.einsum("pqab,map,nbq->mn", P, SIG, SIG)


@pytest.mark.parametrize("ch", range(5))
def test_channel_table_matches_spin_tensor_product(tables, ch):
    terms, _ = tables
    assert len(terms[ch]) == 256
    rng = np.random.default_rng(ch)
    for _ in range(4):
        ra, rb = rng.normal(size=(4, 4)), rng.normal(size=(4, 4))
        ga, gb = np.where(XIXI > 0, 1.0, 1j) * ra, np.where(XIXI > 0, 1.0, 1j) * rb
        form, sign = FORMS[ch]
        out = _basis(sign * np.einsum(form, _tensor(ga), _tensor(gb)))
        keep = np.where(XIXI > 0, out.real, out.imag)
        drop = np.where(XIXI > 0, out.imag, out.real)
        acc = np.zeros(16)
        for c1, c2, q, k in terms[ch]:
            acc[q] += k * ra.flat[c1] * rb.flat[c2]
        assert np.abs(acc.reshape(4, 4) - keep).max() <= 1e-13
        assert np.abs(drop).max() <= 1e-13


def test_every_input_pair_feeds_one_output(tables):
    terms, _ = tables
    for ch in range(4):
        assert all(k in (1, -1) for _, _, _, k in terms[ch])
    rpa = [(c1, c2, k) for c1, c2, _, k in terms[4] if k != 0]
    assert len(rpa) == 64 and all(c1 % 4 == c2 // 4 and k in (2, -2) for c1, c2, k in rpa)


def test_correlation_exchange_coefficients(tables):
    """Re of sum sigma^mu_{a1 a1'} sigma^nu_{a2 a2'} X[a1'][a2'][a1][a2] with
    X[a1'][a2'][a1][a2] = V[a2'][a1'][a1][a2] (the legs 1' and 2' exchanged)
    for a unit basis function Gamma^{mu' nu'} in the real representation."""
    _, chi_x = tables
    for qp in range(16):
        G = np.zeros((4, 4), dtype=complex)
        G.flat[qp] = 1.0 if XIXI.flat[qp] > 0 else 1j
        V = _tensor(G)
        X = np.einsum("qpab->pqab", V)
        for m in range(16):
            mu, nu = divmod(m, 4)
            v = np.einsum("ap,bq,pqab->", SIG[mu], SIG[nu], X)
            assert abs(chi_x[m, qp] - v.real) <= 1e-13, (m, qp)
