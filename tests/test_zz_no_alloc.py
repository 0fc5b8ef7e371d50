"""pffrg_chi_noalloc (no context, no device allocation) against pffrg_chi.

Two calls in a row through the C ABI, the second on a smaller problem
(fewer frequencies and pairs), each compared with the context entry point
pffrg_chi on the same state: the two run the same kernels on the same
inputs, so the results must agree bit for bit (and with the FP64 oracle to
1e-10).  The fixed scratch area keeps the first call's contents when the
second one runs; a result that depended on them would differ.
"""

import ctypes

import numpy as np
import pytest

import workloads as W
from tests.parity import compare_chi, expand_state

pytestmark = pytest.mark.gpu

CASES = [("honeycomb", dict(j1=1.0, j2=0.4, j3=0.2), 3, W.log_mesh(0.01, 30.0, 10), 0.31, 7),
         ("square", dict(j1=1.0, j2=0.5), 2, W.log_mesh(0.02, 20.0, 6), 0.47, 8)]


def test_chi_noalloc_matches_context_chi_twice_shrinking():
    import torch
    import oracle
    from paper_2109_13317_amd import _lib, build_tables
    from paper_2109_13317_amd.flow import Context
    lib = _lib.load()
    sizes = []
    for lat, params, L, mesh, lam, seed in CASES:
        model = W.model(lat, **params)
        tables = build_tables(model, L)
        ctx = Context(tables, mesh)
        nf, ns = ctx.nf, ctx.ns
        sizes.append((nf, ns))
        print(f"no-alloc chi: {lat} range {L}, {nf} frequencies, {ns} pairs, lambda {lam}", flush=True)
        x = torch.from_numpy(W.random_state(nf, ns, seed=seed, scale=0.2)).cuda()
        ref = ctx.chi(lam, x).clone()
        d_w = torch.from_numpy(np.ascontiguousarray(mesh, dtype=np.float64)).cuda()
        d_sw = torch.from_numpy(np.ascontiguousarray(tables.swap, dtype=np.int32)).cuda()
        out = torch.full((2 * ns,), float("nan"), dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream()
        _lib.check(lib.pffrg_chi_noalloc(nf, ctypes.c_void_p(d_w.data_ptr()), ns, ctypes.c_void_p(d_sw.data_ptr()),
                                         float(lam), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(stream.cuda_stream)))
        torch.cuda.synchronize()
        assert torch.equal(out.view(2, ns), ref), (out, ref)
        orc = oracle.Oracle(model, L, mesh)
        zz, dd = orc.chi(lam, expand_state(orc, tables, x.cpu().numpy()))
        assert compare_chi(orc, tables, zz, dd, out.cpu().numpy()) <= 1e-10
    assert sizes[1][0] < sizes[0][0] and sizes[1][1] < sizes[0][1]
