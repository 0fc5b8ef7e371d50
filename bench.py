#!/usr/bin/env python3
"""Benchmark of the SU(2) pf-FRG flow hot path on one MI355X.

Headline workload: pyrochlore nearest-neighbour Heisenberg model (fcc lattice
with the four-site tetrahedral basis), vertex range 5 bonds (31
symmetry-reduced pairs, 277 sites in range), 48 positive Matsubara
frequencies log-spaced 1e-3..100, FP64: the largest FP64 configuration of the
benchmark set on one GPU (3.5 M vertex elements, 28 MB state).  Synthetic
input: the flow state is the physical flow from the initial condition
(Lambda 100 -> 1 in 40 RK4 steps, untimed setup); no datasets or trained
weights are involved.

One timed step = one pass of the whole hot path: a classical RK4 step
(4 self-energy + 4 vertex right-hand sides and the stage combinations) from
Lambda to 0.95 Lambda, then chi per pair and chi(k) on 16^3 k-points.
`value` = vertex-RHS elements per second = 4 * E / step time, with
E = 2 * pairs * triples vertex elements per right-hand side.

Also reported: the dominant kernel's roofline position (algorithmic FP64
flops per launch over its HIP-event duration), the whole flows of the
headline workload (fixed RK4 on the exponential schedule b = 0.95, and the
adaptive Dormand-Prince 5(4) flow with chi(k) every accepted step), the CPU
oracle timed on a bounded sample of the same workload, and, as extras, the
square J1-J2 workload's hot path and adaptive flow (range 7, 32
frequencies), the FP32 mode, a 64-point phase scan advanced as one batch
against 64 sequential FP64 flows, d chi(k_peak)/dJ through a 120-step flow
by the discrete adjoint against the forward cost, and the growth of the
vertex right-hand side with the frequency and pair counts.  paper_context
quotes the only throughput the paper allows to derive (a CPU node, another
workload): context, not a baseline.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

PEAK_FP64_VECTOR_TFLOPS = 78.6     # 256 CU x 2.4 GHz x 128 FP64 flop/clk/CU
PEAK_HBM_GBS = 8000.0

# HBM bytes per timed vertex launch from the two rocprofv3 --pmc runs
# (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, copy-kernel calibrated): the
# k_vertex_stu launch up to 20 pairs, the whole concurrent vertex right-hand
# side beyond (k_vertex_t, both k_vertex_su launches and the t-part sum);
# keyed by the hash of the kernel sources they were taken on and the
# workload; a changed kernel reports traffic null until the counters are
# taken again.
MEASURED_TRAFFIC = {
    ("351b2e87dc4c0019", "pyrochlore"): 277.63e6,
}


def kernel_source_hash() -> str:
    """Hash of the vertex kernel sources with comments and blank lines removed
    (an edit of a comment keeps the recorded counters)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("kernels_flow.h", "device_common.h"):
        with open(os.path.join(ROOT, "paper_2109_13317_amd", "csrc", f)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def log(*a):
    print(f"[bench {time.strftime('%H:%M:%S')}]", *a, file=sys.stderr, flush=True)


def node_counts(mesh: np.ndarray, lam: float) -> np.ndarray:
    """Evaluation points per channel (s, t, u) and transfer frequency index:
    delta points of the single-scale propagator plus trapezoid nodes of the
    Katanin domain (same rule as the kernels; counting only)."""
    nf = len(mesh)
    wmax = mesh[-1]
    full = np.concatenate([-mesh[::-1], mesh])
    out = np.zeros((3, nf), dtype=np.int64)
    for ch in range(3):
        for iv, nu in enumerate(mesh):
            n = 0
            for x in (lam, -lam):
                winv = nu - x if ch == 0 else (x + nu if ch == 1 else x - nu)
                px = nu - x if ch == 0 else (x - nu if ch == 1 else nu + x)
                n += int(abs(winv) >= lam) + int(abs(px) >= lam)
            c = nu if ch < 2 else -nu
            e0, e1 = c - lam, c + lam
            for a, b in ((-wmax, -lam), (lam, wmax)):
                if not a < b:
                    continue
                for lo, hi in ((a, min(b, e0)), (max(a, e1), b)):
                    if lo < hi:
                        n += 2 + int(np.count_nonzero((full > lo) & (full < hi)))
            out[ch, iv] = n
    return out


def checkpoint_cost(x) -> dict:
    """Time to write and read back one flow snapshot of state x (median of 3,
    a temporary directory on the host's disk)."""
    import tempfile
    import torch
    from paper_2109_13317_amd import checkpoint as ck
    state = x.cpu().numpy()
    wr, rd = [], []
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "flow.checkpoint")
        for _ in range(3):
            t0 = time.perf_counter()
            torch.cuda.synchronize()
            ck.write(p, x.cpu().numpy(), {"format": ck.FORMAT})
            wr.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            x.copy_(torch.from_numpy(ck.read(p).state))
            torch.cuda.synchronize()
            rd.append(time.perf_counter() - t0)
        size = os.path.getsize(p)
    assert (x.cpu().numpy() == state).all()
    return {"bytes": size, "write_ms": 1e3 * float(np.median(wr)), "read_ms": 1e3 * float(np.median(rd)),
            "includes": "device-host copy, npz write with fsync and rename / read and host-device copy"}


def vertex_flops(mesh: np.ndarray, lam: float, ns: int, n_terms: int) -> dict:
    """Algorithmic FP64 flops of one vertex right-hand side at cutoff lam,
    per channel launch.

    Per triple (s,t,u) with n_s, n_t, n_u evaluation points:
      s and u channels: 45 flops per pair and point (two interpolated vertex
      vectors, 2 strains x 4 corners FMA = 16 flops each, and 13 flops of
      channel products and accumulation);
      t channel: 52 flops per pair and point (two vectors and 20 flops of the
      two vertex corrections), 32 flops per point for the two on-site
      vertices, 4 ns^2 flops per point for the lattice-sum matrix (two
      strains, GEMM form) and 4 flops per tabulated term.
    """
    nc = node_counts(mesh, lam)
    nf = len(mesh)
    out = {"s": 0.0, "u": 0.0, "t": 0.0}
    for a in range(nf):
        for c in range(a + 1):
            for t in range(nf):
                out["s"] += 45.0 * ns * nc[0, a]
                out["u"] += 45.0 * ns * nc[2, c]
                nt = nc[1, t]
                out["t"] += 52.0 * ns * nt + 4.0 * ns * ns * nt + 32.0 * nt + 4.0 * n_terms
    out["all"] = out["s"] + out["u"] + out["t"]
    return out


def xyz_vertex_flops(mesh: np.ndarray, lam: float, ns: int, n_terms: int) -> float:
    """Algorithmic FP64 flops of one XYZ vertex right-hand side at cutoff lam
    (four strains).  Per triple and evaluation point:
      s and u: 100 flops per pair (two interpolated vectors, 4 strains x 4
      corners FMA = 32 flops each, and 36 flops of channel products);
      t: 148 flops per pair (the two vectors, the two vertex corrections of
      every strain with their 4-term sign sums, the weighted site vector),
      64 flops for the two on-site vertices, 8 ns^2 for the four lattice-sum
      matrices (GEMM form), and 8 flops per tabulated term."""
    nc = node_counts(mesh, lam)
    nf = len(mesh)
    tot = 0.0
    for a in range(nf):
        for c in range(a + 1):
            for t in range(nf):
                tot += 100.0 * ns * (nc[0, a] + nc[2, c])
                nt = nc[1, t]
                tot += 148.0 * ns * nt + 8.0 * ns * ns * nt + 64.0 * nt + 8.0 * n_terms
    return tot


def tri_vertex_flops(mesh: np.ndarray, lam: float, ns: int, n_terms: int) -> dict:
    """Algorithmic FP64 flops of one general (TRI, sixteen-component) vertex
    right-hand side at cutoff lam, per channel.  Per triple and evaluation
    point:
      s and u: 768 flops per pair (two interpolated vertices, 16 components x
      4 corners FMA = 128 flops each, and the channel product, 256 FMA);
      t: 1280 flops per pair (the two vertices and the two vertex corrections,
      256 FMA each), 256 flops for the two on-site vertices, and the lattice
      sum term by term: 64 FMA (sum_k Gamma_a^{mu k} Gamma_b^{k nu}) per
      tabulated term."""
    nc = node_counts(mesh, lam)
    nf = len(mesh)
    out = {"s": 0.0, "u": 0.0, "t": 0.0}
    for a in range(nf):
        for c in range(a + 1):
            for t in range(nf):
                out["s"] += 768.0 * ns * nc[0, a]
                out["u"] += 768.0 * ns * nc[2, c]
                nt = nc[1, t]
                out["t"] += (1280.0 * ns + 256.0 + 128.0 * n_terms) * nt
    out["all"] = out["s"] + out["u"] + out["t"]
    return out


def gather_instructions(mesh: np.ndarray, lam: float, ns: int) -> float:
    """Wave-level 16-byte vertex gathers of one FP64 vertex right-hand side
    (counting only): lanes cover G = 64 // ns evaluation points of one triple
    at once, each point reads the four corners of two interpolated vectors;
    the t channel takes its points in sub-chunks of 4 (8 at 17-20 pairs) and
    reads the two on-site vertices (four corners each) once per 16 points."""
    nc = node_counts(mesh, lam)
    nf = len(mesh)
    G = max(1, 64 // ns)
    sub = 8 if 16 < ns <= 20 else 4
    tot = 0.0
    for a in range(nf):
        for c in range(a + 1):
            for t in range(nf):
                tot += 8 * math.ceil(nc[0, a] / G) + 8 * math.ceil(nc[2, c] / G)
                nt = int(nc[1, t])
                full, rest = divmod(nt, sub)
                tot += 8 * (full * math.ceil(sub / G) + (math.ceil(rest / G) if rest else 0))
                tot += 4 * math.ceil(nt / 16)
    return tot


def kgrid(n: int) -> np.ndarray:
    m = (np.arange(n) / n - 0.5) * 2 * math.pi
    kx, ky = np.meshgrid(m, m, indexing="ij")
    return np.stack([kx.ravel(), ky.ravel(), np.zeros(n * n)], axis=1)


def fp32_leg(tables, wl, x_np, lam, reps=10):
    """The same right-hand side in FP32 mode (vertex gathers, products and
    lattice-sum matrix in FP32 with compensated sums) next to FP64."""
    import torch
    from paper_2109_13317_amd.flow import Context
    x = torch.from_numpy(x_np).cuda()
    res = {}
    for prec in ("fp64", "fp32"):
        c = Context(tables, wl.mesh, precision=prec)
        out = c.new_state()
        c.rhs(lam, x, out)
        torch.cuda.synchronize()
        c.set_profiling(True, kernels=("vertex",))
        for _ in range(reps):
            c.rhs(lam, x, out)
        ms, n = c.profile_read("vertex")
        c.set_profiling(False)
        res[prec] = (ms / n, out.cpu().numpy())
    nf = len(wl.mesh)
    a, b = res["fp64"][1], res["fp32"][1]
    E = a.size - nf
    return {"vertex_rhs_ms": res["fp32"][0], "vertex_rhs_ms_fp64": res["fp64"][0],
            "vertex_rhs_elements_per_s": E / (res["fp32"][0] * 1e-3),
            "speedup_vs_fp64": res["fp64"][0] / res["fp32"][0],
            "max_rel_err_vs_fp64": float(np.abs(a[nf:] - b[nf:]).max() / np.abs(a[nf:]).max()),
            "sigma_part": "FP64 in both (bitwise equal)" if np.array_equal(a[:nf], b[:nf]) else "differs",
            "lambda": lam}


def _fp64_steps(ctx, sched, kp):
    """A plain FP64 flow along sched one step at a time (untimed): per step
    the cutoff, chi, max chi(k) over kp and max |vertex|; stops at the first
    step whose state is not finite (the library restores the last finite
    state and reports it)."""
    import torch
    from paper_2109_13317_amd._lib import PffrgError
    x = ctx.init_state()
    rec = []
    for i in range(len(sched) - 1):
        try:
            ctx.flow(x, schedule=sched[i:i + 2], scheme="rk4")
        except PffrgError:
            break
        chi = ctx.chi(sched[i + 1], x)
        rec.append((sched[i + 1], chi.cpu().numpy(), float(ctx.chi_k(chi.reshape(-1), kp).max()),
                    float(torch.abs(x[ctx.nf:]).max())))
    return rec


def batch_leg():
    """64-point square J1-J2 scan (J2/J1 = k/63, ranges 4..7, 24 frequencies),
    RK4 100 -> 0.01 in 120 steps: one FP32 batch (persistent vertex launch,
    hipGraph step, tuned launch shape) against 64 sequential plain FP64 flows
    (both timed), then both again step by step (untimed) for every point's
    breakdown, last finite cutoff and chi error against FP64."""
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Batch, Context
    from paper_2109_13317_amd._lib import PffrgError
    from paper_2109_13317_amd.breakdown import batch_breakdowns, find_breakdown
    wl = W.workload("square_scan")
    pts = W.batch_scan_points(64)
    tables = [build_tables(W.model("square", j1=q["j1"], j2=q["j2"]), q["range"]) for q in pts]
    sched = [float(v) for v in wl.schedule]
    lam_max = wl.mesh[-1] / 4
    b = Batch(tables, wl.mesh, precision="fp32")
    x = b.init_state()
    tuned = b.tune(0.5, x)
    x = b.init_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok = b.flow(x, sched, use_graph=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batch scan flow {t_batch:.3f} s ({sum(ok)} of 64 points finite)")
    seq_ok = []
    t_seq = 0.0
    for t in tables:
        c = Context(t, wl.mesh)
        xs = c.init_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            c.flow(xs, schedule=sched, scheme="rk4")
            fin = True
        except PffrgError:
            fin = False
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        seq_ok.append(fin)
        c.close()
    log(f"64 sequential FP64 flows {t_seq:.3f} s ({sum(seq_ok)} of 64 points finite)")
    # untimed: both again step by step; chi(k) on 32 x 32 points after every
    # step for the breakdown detector (a kink or divergence of chi_max(Lambda))
    g = 2 * np.pi * (np.arange(32) / 32 - 0.5)
    kx, ky = np.meshgrid(g, g, indexing="ij")
    kp32 = torch.from_numpy(np.stack([kx.ravel(), ky.ravel(), np.zeros(kx.size)], 1).copy()).cuda()
    rec32 = []
    bds, lams, _ = batch_breakdowns(b, b.init_state(), sched, kp32, lam_max=lam_max, record=rec32)
    b.close()
    points = []
    for p, (q, t) in enumerate(zip(pts, tables)):
        c = Context(t, wl.mesh)
        r64 = _fp64_steps(c, sched, kp32)
        c.close()
        n64 = len(r64)                       # finite FP64 steps
        n32 = 0                              # finite FP32 steps (the state stays non-finite once it is)
        while n32 < len(rec32) and rec32[n32][1][p]:
            n32 += 1
        bd64 = find_breakdown([r[0] for r in r64], [r[2] for r in r64], lam_max=lam_max)
        # the last step above either precision's breakdown (or the last step
        # both finished) is where FP32 must still follow FP64
        stops = [n64, n32] + [bd.index for bd in (bd64, bds[p]) if bd.index is not None]
        ref = min(stops) - 1
        err = None
        if ref >= 0:
            a64, a32 = r64[ref][1], rec32[ref][2][p]
            err = float(np.abs(a32 - a64).max() / np.abs(a64).max())
        d = {"j2_over_j1": q["j2"] / q["j1"], "range": q["range"], "pairs": t.n_pairs,
             "breakdown_fp64": {"kind": bd64.kind, "lambda": bd64.lam},
             "breakdown_fp32": {"kind": bds[p].kind, "lambda": bds[p].lam},
             "last_finite_lambda_fp64": r64[-1][0] if n64 else sched[0],
             "last_finite_lambda_fp32": rec32[n32 - 1][0] if n32 else sched[0],
             "chi_rel_err_at_last_lambda_above_breakdown": err,
             "lambda_of_that_step": r64[ref][0] if ref >= 0 else None}
        if n32 < n64:
            # a point that FP64 carries further than FP32: the FP64 vertex size
            # and the chi disagreement at the last step both finished
            d["lost_to_fp32"] = {
                "fp64_max_abs_vertex_at_fp32_loss": r64[n32][3] if n32 < n64 else None,
                "fp64_max_abs_vertex_before": r64[n32 - 1][3] if n32 else None,
                "chi_rel_diff_at_last_common_step": (float(np.abs(rec32[n32 - 1][2][p] - r64[n32 - 1][1]).max()
                                                          / np.abs(r64[n32 - 1][1]).max()) if n32 else None)}
        points.append(d)
    errs = [d["chi_rel_err_at_last_lambda_above_breakdown"] for d in points
            if d["chi_rel_err_at_last_lambda_above_breakdown"] is not None]
    lost = [d for d in points if "lost_to_fp32" in d]
    below = sum(1 for d in lost if d["breakdown_fp64"]["lambda"] is not None
                and d["last_finite_lambda_fp32"] < d["breakdown_fp64"]["lambda"])
    log(f"batch scan: chi error at the last step above breakdown max {max(errs):.2e} over {len(errs)} points; "
        f"{len(lost)} points finite further in FP64 than in FP32, {below} of them lost below the FP64 breakdown")
    for d in lost:
        log(f"  J2/J1 {d['j2_over_j1']:.3f} range {d['range']}: FP32 last finite {d['last_finite_lambda_fp32']:.4g}, "
            f"FP64 {d['last_finite_lambda_fp64']:.4g}, breakdown {d['breakdown_fp64']}, "
            f"{d['lost_to_fp32']}")
    return {"workload": "64 square J1-J2 points, J2/J1 = k/63, ranges 4..7 (9/12/16/20 pairs), 24 log freqs "
                        "1e-3..100, RK4 100 -> 0.01 in 120 steps",
            "batch_fp32_seconds": t_batch, "sequential_fp64_seconds": t_seq,
            "speedup": t_seq / t_batch, "tuned_launch": {"per_xcd": tuned[0], "order": tuned[1], "split": tuned[2]},
            "finite_points_batch": int(sum(ok)), "finite_points_fp64": int(sum(seq_ok)),
            "sequential_note": "a diverging FP64 flow stops at its first non-finite step",
            "chi_rel_err_at_last_lambda_above_breakdown": {"points": len(errs), "max": max(errs),
                                                           "median": float(np.median(errs))},
            "points_finite_further_in_fp64": len(lost), "of_them_lost_below_fp64_breakdown": below,
            "points": points,
            "method": "untimed step-by-step passes of both: chi(k) on 32 x 32 points after every RK4 step, "
                      "breakdown = first kink or divergence of chi_max(Lambda) below a quarter of the top mesh "
                      "frequency (breakdown.find_breakdown); chi error = max |chi_fp32 - chi_fp64| / max "
                      "|chi_fp64| over pairs and both strains at the last step above the earlier breakdown "
                      "of the two (or the last step both finished)"}


def adjoint_leg():
    """d chi(k_peak, Lambda=0.1) / d(J1, J2, J3) on the honeycomb lattice
    (range 6, 32 frequencies, RK4 100 -> 0.1 in 120 steps) through the
    discrete adjoint, timed against the forward flow, and checked against
    central differences of the forward flow."""
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import ChiAdjoint, Context
    wl = W.workload("honeycomb_j123")
    shells = ("j1", "j2", "j3")
    J0 = np.array([wl.params[s] for s in shells])
    D = np.stack([build_tables(W.model("honeycomb", **{s: 1.0}), wl.range).coupling for s in shells], axis=1)
    ctx = Context(build_tables(wl.model(), wl.range), wl.mesh)
    sched = wl.schedule
    grid = torch.from_numpy(kgrid(64)).cuda()
    x = ctx.init_state()
    ctx.flow(x, schedule=sched, scheme="rk4")
    ck = ctx.chi_k(ctx.chi(sched[-1], x), grid)
    kpk = grid[int(torch.argmax(ck))].reshape(1, 3).cpu()
    x = ctx.init_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.flow(x, schedule=sched, scheme="rk4")
    ctx.chi_k(ctx.chi(sched[-1], x), kpk.cuda())
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    J = torch.tensor(J0, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = ChiAdjoint.apply(J, ctx, D, sched, kpk)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out.sum().backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    grad = J.grad.numpy()
    log(f"adjoint: forward {t_fwd:.3f} s, checkpointed forward {t1 - t0:.3f} s, backward {t2 - t1:.3f} s "
        f"({(t2 - t0) / (6.0 * t_fwd):.2f} x the 6 forward flows of central differences in 3 couplings)")

    def f(jv):
        xx = ctx.init_state_from(D @ jv)
        ctx.flow(xx, schedule=sched, scheme="rk4")
        return float(ctx.chi_k(ctx.chi(sched[-1], xx), kpk.cuda()).cpu()[0])

    fd = np.zeros(3)
    for i in range(3):
        def cd(h):
            e = np.zeros(3); e[i] = h
            return (f(J0 + e) - f(J0 - e)) / (2 * h)
        h = 1e-3 * abs(J0[i])
        fd[i] = (4.0 * cd(h / 2) - cd(h)) / 3.0
    return {"workload": "honeycomb J1-J2-J3 (J from default_rng(210913317)), range 6 (14 pairs), 32 log freqs, "
                        "RK4 100 -> 0.1 in 120 steps, k_peak = argmax chi(k) on 64x64",
            "J": J0.tolist(), "k_peak": kpk.numpy().ravel().tolist(), "chi_k_peak": float(out.detach()[0]),
            "dchi_dJ": grad.tolist(), "forward_seconds": t_fwd, "checkpointed_forward_seconds": t1 - t0,
            "adjoint_seconds": t2 - t1, "adjoint_over_forward": (t1 - t0 + t2 - t1) / t_fwd,
            "adjoint_over_central_differences_3_couplings": (t2 - t0) / (6.0 * t_fwd),
            "checkpoint_bytes": int((len(sched) - 1) * ctx.size * 8),
            "central_differences_equivalent": {
                "flows_for_3_shell_couplings": 6, "flows_for_per_pair_couplings": 2 * (ctx.ns - 1),
                "note": "the adjoint returns d chi/d J for every pair coupling at once (ratio above, in forward "
                        "flows); central differences need two flows per parameter (off-site pairs only: the on-site pair has no coupling)"},
            "fd_check": {"method": "central differences of the forward flow, h = 1e-3 J_i, Richardson",
                         "max_rel_err": float(np.abs(grad - fd).max() / np.abs(fd).max())}}


def xyz_leg(reps=10):
    """XYZ flow (Sec. 2, diagonal vertex components): honeycomb J1-J2-J3 with
    (Jx, Jy, Jz) couplings per shell, range 6 (14 pairs), 32 log frequencies
    1e-3..100: one right-hand side at Lambda = 0.5 on the flowed state (HIP
    events around the vertex launches) and the RK4 flow 100 -> 0.1 in 120
    steps, beside the SU(2) flow of the same lattice and mesh."""
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    model = W.model_xyz("honeycomb", j1=(0.9, 0.7, 0.5), j2=(0.3, 0.2, 0.25), j3=(0.1, 0.15, 0.3))
    mesh = W.log_mesh(1e-3, 100.0, 32)
    tables = build_tables(model, 6)
    sched = W.geometric_schedule(100.0, 0.1, 120)
    res = {"workload": "XYZ honeycomb J1-J2-J3, J1 = (0.9, 0.7, 0.5), J2 = (0.3, 0.2, 0.25), J3 = (0.1, 0.15, "
                       "0.3), range 6 (14 pairs), 32 log freqs 1e-3..100; RK4 100 -> 0.1 in 120 steps"}
    for sym, tab in (("xyz", tables), ("su2", build_tables(W.model("honeycomb", j1=0.9, j2=0.3, j3=0.1), 6))):
        ctx = Context(tab, mesh)
        x = ctx.init_state()
        ctx.flow(x, schedule=[l for l in sched if l >= 0.5], scheme="rk4")
        out = ctx.new_state()
        ctx.rhs(0.5, x, out)
        ctx.set_profiling(True, kernels=("vertex",))
        for _ in range(reps):
            ctx.rhs(0.5, x, out)
        ms, n = ctx.profile_read("vertex")
        ctx.set_profiling(False)
        xf = ctx.init_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.flow(xf, schedule=sched, scheme="rk4")
        torch.cuda.synchronize()
        t_flow = time.perf_counter() - t0
        E = ctx.nc * ctx.ns * ctx.nf * ctx.nf * (ctx.nf + 1) // 2
        r = {"vertex_rhs_ms": ms / n, "vertex_elements": E, "elements_per_s": E / (ms / n * 1e-3),
             "flow_seconds": t_flow}
        if sym == "xyz":
            fl = xyz_vertex_flops(mesh, 0.5, ctx.ns, tab.n_terms)
            r.update({"flops": fl, "tflops": fl / (ms / n * 1e-3) / 1e12,
                      "frac_of_fp64_peak": fl / (ms / n * 1e-3) / 1e12 / PEAK_FP64_VECTOR_TFLOPS})
        res[sym] = r
        ctx.close()
    res["xyz_over_su2_rhs_time"] = res["xyz"]["vertex_rhs_ms"] / res["su2"]["vertex_rhs_ms"]
    # bond-dependent couplings beyond 16 pairs (the four-waves-per-triple t
    # channel): Heisenberg-Kitaev honeycomb, range 4 (31 pairs)
    hk = W.model_heisenberg_kitaev(1.0, -2.0)
    tab = build_tables(hk, 4)
    hk_res = {"workload": "Heisenberg-Kitaev honeycomb J = 1, K = -2, range 4 (31 pairs: no lattice symmetry maps "
                          "one bond direction onto another), 32 log freqs 1e-3..100, RHS at Lambda = 0.5 on a seeded "
                          "random state"}
    for prec in ("fp64", "fp32"):
        ctx = Context(tab, mesh, precision=prec)
        x = torch.from_numpy(W.random_state(ctx.nf, ctx.ns, seed=7, scale=0.2, strains=4)).cuda()
        out = ctx.new_state()
        ctx.rhs(0.5, x, out)
        ctx.set_profiling(True, kernels=("vertex",))
        for _ in range(reps):
            ctx.rhs(0.5, x, out)
        ms, n = ctx.profile_read("vertex")
        ctx.set_profiling(False)
        fl = xyz_vertex_flops(mesh, 0.5, ctx.ns, tab.n_terms)
        E = ctx.nc * ctx.ns * ctx.nf * ctx.nf * (ctx.nf + 1) // 2
        r = {"vertex_rhs_ms": ms / n, "vertex_elements": E, "elements_per_s": E / (ms / n * 1e-3), "flops": fl,
             "tflops": fl / (ms / n * 1e-3) / 1e12}
        if prec == "fp64":
            r["frac_of_fp64_peak"] = r["tflops"] / PEAK_FP64_VECTOR_TFLOPS
            hk_res.update(r)
        else:
            hk_res["fp32"] = r
        ctx.close()
    hk_res["fp32_speedup"] = hk_res["vertex_rhs_ms"] / hk_res["fp32"]["vertex_rhs_ms"]
    res["heisenberg_kitaev_range4"] = hk_res
    log(f"XYZ Heisenberg-Kitaev range 4 ({tab.n_pairs} pairs): vertex RHS {hk_res['vertex_rhs_ms']:.3f} ms "
        f"({hk_res['tflops']:.2f} TFLOP/s), FP32 {hk_res['fp32']['vertex_rhs_ms']:.3f} ms "
        f"({hk_res['fp32_speedup']:.2f}x)")
    log(f"XYZ: vertex RHS {res['xyz']['vertex_rhs_ms']:.3f} ms ({res['xyz']['tflops']:.2f} TFLOP/s), SU(2) "
        f"{res['su2']['vertex_rhs_ms']:.3f} ms; flows {res['xyz']['flow_seconds']:.3f} / "
        f"{res['su2']['flow_seconds']:.3f} s")
    return res


def tri_leg(reps=5):
    """General (TRI) flow (Sec. 2 general couplings, all sixteen vertex
    components): Kitaev-Gamma honeycomb (J = 0.2, K = -1, G = 0.5), range 4
    (31 pairs), 32 log frequencies 1e-3..100: one right-hand side at
    Lambda = 0.5 on a seeded random state (HIP events around the vertex
    launches), next to the XYZ (Heisenberg-Kitaev, the same bonds and pairs)
    and SU(2) contexts of the same lattice and mesh, and a 20-step RK4 flow
    from Lambda = 100."""
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    mesh = W.log_mesh(1e-3, 100.0, 32)
    lam = 0.5
    res = {"workload": "Kitaev-Gamma honeycomb J = 0.2, K = -1, G = 0.5, range 4 (31 pairs), 32 log freqs "
                       "1e-3..100, RHS at Lambda = 0.5 on a seeded random state"}
    models = (("tri", W.model_kitaev_gamma(0.2, -1.0, 0.5), 16),
              ("xyz", W.model_heisenberg_kitaev(0.2, -1.0), 4),
              ("su2", W.model("honeycomb", j1=0.2), 2))
    for name, model, strains in models:
        tab = build_tables(model, 4)
        ctx = Context(tab, mesh)
        x = torch.from_numpy(W.random_state(ctx.nf, ctx.ns, seed=7, scale=0.2, strains=strains)).cuda()
        out = ctx.new_state()
        ctx.rhs(lam, x, out)
        ctx.set_profiling(True, kernels=("vertex",))
        for _ in range(reps):
            ctx.rhs(lam, x, out)
        ms, n = ctx.profile_read("vertex")
        ctx.set_profiling(False)
        E = ctx.nc * ctx.ns * ctx.nf * ctx.nf * (ctx.nf + 1) // 2
        r = {"pairs": ctx.ns, "vertex_rhs_ms": ms / n, "vertex_elements": E, "elements_per_s": E / (ms / n * 1e-3)}
        if name == "tri":
            fl = tri_vertex_flops(mesh, lam, ctx.ns, tab.n_terms)
            r.update({"flops": fl["all"], "flops_by_channel": {k: fl[k] for k in ("s", "u", "t")},
                      "tflops": fl["all"] / (ms / n * 1e-3) / 1e12,
                      "frac_of_fp64_peak": fl["all"] / (ms / n * 1e-3) / 1e12 / PEAK_FP64_VECTOR_TFLOPS,
                      "n_terms": tab.n_terms})
            xf = ctx.init_state()
            sched = W.geometric_schedule(100.0, 100.0 * 0.9 ** 20, 20)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.flow(xf, schedule=sched, scheme="rk4")
            torch.cuda.synchronize()
            r["rk4_20_steps_seconds"] = time.perf_counter() - t0
        res[name] = r
        ctx.close()
    # the same model with the joint lattice and spin transformations of Sec. 4.1
    tab = build_tables(models[0][1], 4, spin_permutations=True)
    ctx = Context(tab, mesh)
    xo = ctx.init_state()
    ctx.flow(xo, schedule=W.geometric_schedule(100.0, lam, 40), scheme="rk4")
    out = ctx.new_state()
    ctx.rhs(lam, xo, out)
    ctx.set_profiling(True, kernels=("vertex",))
    for _ in range(reps):
        ctx.rhs(lam, xo, out)
    ms, n = ctx.profile_read("vertex")
    ctx.set_profiling(False)
    fl = tri_vertex_flops(mesh, lam, ctx.ns, tab.n_terms)
    res["tri_spin_permutations"] = {
        "pairs": ctx.ns, "n_terms": tab.n_terms, "rotations": len(tab.rot), "vertex_rhs_ms": ms / n,
        "state": "flowed from Lambda = 100 in 40 RK4 steps (a state with the model's symmetries)",
        "flops": fl["all"], "tflops": fl["all"] / (ms / n * 1e-3) / 1e12,
        "speedup_vs_lattice_symmetries_only": res["tri"]["vertex_rhs_ms"] / (ms / n)}
    ctx.close()
    res["tri_over_xyz_rhs_time"] = res["tri"]["vertex_rhs_ms"] / res["xyz"]["vertex_rhs_ms"]
    res["tri_over_su2_rhs_time"] = res["tri"]["vertex_rhs_ms"] / res["su2"]["vertex_rhs_ms"]
    log(f"TRI Kitaev-Gamma range 4 ({res['tri']['pairs']} pairs): vertex RHS {res['tri']['vertex_rhs_ms']:.3f} ms "
        f"({res['tri']['tflops']:.2f} TFLOP/s, {res['tri']['frac_of_fp64_peak']:.3f} of FP64 peak); XYZ "
        f"{res['xyz']['vertex_rhs_ms']:.3f} ms, SU(2) {res['su2']['vertex_rhs_ms']:.3f} ms; with spin permutations "
        f"{res['tri_spin_permutations']['pairs']} pairs, {res['tri_spin_permutations']['vertex_rhs_ms']:.3f} ms")
    return res


def scaling_leg(lam=0.7, reps=5):
    """Vertex right-hand-side time against the frequency count (square J1-J2,
    range 7) and against the pair count (square J1-J2, ranges 4..7, 32
    frequencies), with the fitted exponents."""
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context

    def t_vertex(tables, nf):
        mesh = W.log_mesh(1e-3, 100.0, nf)
        c = Context(tables, mesh)
        x = torch.from_numpy(W.random_state(nf, c.ns, seed=1, scale=0.2)).cuda()
        out = c.new_state()
        c.rhs(lam, x, out)
        torch.cuda.synchronize()
        c.set_profiling(True, kernels=("vertex",))
        for _ in range(reps):
            c.rhs(lam, x, out)
        ms, n = c.profile_read("vertex")
        c.close()
        return ms / n

    model = W.model("square", j1=1.0, j2=0.5)
    t7 = build_tables(model, 7)
    nfs = [16, 24, 32, 48]
    tn = [t_vertex(t7, nf) for nf in nfs]
    ranges = [4, 5, 6, 7]
    tabs = [build_tables(model, L) for L in ranges]
    tl = [t_vertex(t, 32) for t in tabs]
    nss = [t.n_pairs for t in tabs]
    slope_nf = float(np.polyfit(np.log(nfs), np.log(tn), 1)[0])
    slope_ns = float(np.polyfit(np.log(nss), np.log(tl), 1)[0])
    return {"lambda": lam, "vs_n_freq": {"n_freq": nfs, "vertex_ms": tn, "exponent": slope_nf},
            "vs_pairs": {"pairs": nss, "ranges": ranges, "vertex_ms": tl, "exponent": slope_ns},
            "note": "work grows like n_freq^3 * (evaluation points ~ n_freq) and like pairs (channel "
                    "products) to pairs^2 (lattice-sum matrix)"}


def _oracle_sample(orc, tables, xo, lam, target_s, threads):
    nf = orc.nf
    rng = np.random.default_rng(0)
    all_tr = [(a, t, c) for a in range(nf) for c in range(a + 1) for t in range(nf)]
    order = rng.permutation(len(all_tr))
    t0 = time.perf_counter()
    dsig = orc.sigma_rhs(lam, xo)
    t_sig = time.perf_counter() - t0
    first = [all_tr[i] for i in order[:threads]]
    t0 = time.perf_counter()
    orc.vertex_rhs_triples(lam, xo, dsig, first)
    spent = time.perf_counter() - t0
    done = len(first)
    more = int(max(0.0, target_s - spent) / (spent / done))
    more = min(more, len(all_tr) - done)
    if more > 0:
        rest = [all_tr[i] for i in order[done:done + more]]
        t0 = time.perf_counter()
        orc.vertex_rhs_triples(lam, xo, dsig, rest)
        spent += time.perf_counter() - t0
        done += len(rest)
    elems = 2 * tables.n_pairs * done
    return elems / spent, done, len(all_tr), spent, spent / done * len(all_tr) + t_sig


def cpu_baseline(model, wl, tables, x_np, lam, target_s=12.0):
    """The oracle on a bounded sample: every vertex element of a set of
    frequency triples (plus the self-energy flow), timed on the host cores
    (all of them, and one thread); scaled to vertex-RHS elements per second
    of the reduced workload."""
    import oracle
    from tests.parity import expand_state
    threads = os.cpu_count() or 1
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    orc = oracle.Oracle(model, wl.range, wl.mesh, threads=threads)
    xo = expand_state(orc, tables, x_np)
    value, done, total, spent, per_rhs = _oracle_sample(orc, tables, xo, lam, target_s, threads)
    orc1 = oracle.Oracle(model, wl.range, wl.mesh, threads=1)
    v1, d1, _, s1, _ = _oracle_sample(orc1, tables, xo, lam, target_s / 3, 1)
    tiny = _tiny_flows(threads)
    return {
        "value": value,
        "unit": "vertex-RHS elements/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{done} of {total} frequency triples (all elements of each, "
                   f"unreduced lattice), one FP64 RHS at Lambda={lam:.4g}, {spent:.1f} s"),
        "rhs_seconds_extrapolated": per_rhs,
        "single_thread": {"value": v1, "sample": f"{d1} triples, {s1:.1f} s"},
        "square_tiny_flow": tiny,
        "host": host_cpu(),
    }


def host_cpu() -> dict:
    """The host the oracle ran on: logical CPUs, model and current clock
    (from /proc/cpuinfo, where present), and how the oracle was compiled."""
    import oracle
    model, mhz = None, []
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                if k.strip() == "model name" and model is None:
                    model = v.strip()
                elif k.strip() == "cpu MHz":
                    mhz.append(float(v))
    except OSError:
        pass
    return {"logical_cpus": os.cpu_count(), "model": model,
            "mhz_mean": float(np.mean(mhz)) if mhz else None,
            "oracle_build": "gcc " + " ".join(oracle.CFLAGS)}


def _tiny_flows(threads):
    """The whole small flow (square, range 2, 8 frequencies 0.005..50, RK4
    50 -> 0.5 in 40 steps, 160 right-hand sides) on the oracle (all cores and
    one thread) and on the GPU, with the largest relative state difference."""
    import torch
    import oracle
    from tests.parity import restrict_state
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    wl = W.workload("square_tiny")
    model = wl.model()
    tables = build_tables(model, wl.range)
    ctx = Context(tables, wl.mesh)
    x = ctx.init_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.flow(x, schedule=wl.schedule, scheme="rk4")
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    res = {}
    for n in (threads, 1):
        orc = oracle.Oracle(model, wl.range, wl.mesh, threads=n)
        t0 = time.perf_counter()
        xo = orc.flow(wl.schedule, scheme="rk4")
        res[n] = (time.perf_counter() - t0, xo)
    ref = restrict_state(orc, tables, res[1][1])
    got = x.cpu().numpy()
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    return {"workload": "square range 2, 8 log freqs 0.005..50, RK4 50 -> 0.5 in 40 steps (160 RHS)",
            "oracle_seconds_all_cores": res[threads][0], "oracle_seconds_1_thread": res[1][0],
            "cores": threads, "gpu_seconds": t_gpu, "max_rel_state_diff": err}


def kgrid3(n: int, extent: float = 4.0 * math.pi) -> np.ndarray:
    """n^3 Cartesian k-points on [-extent/2, extent/2)^3 (pyrochlore: the
    cubic cell has side 1, so this covers the extended Brillouin zone)."""
    m = (np.arange(n) / n - 0.5) * extent
    kx, ky, kz = np.meshgrid(m, m, m, indexing="ij")
    return np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)


HOT_PATH = {
    # workload, k-grid of chi(k) per step, description
    "pyrochlore": ("pyrochlore NN Heisenberg J=1, range 5 (31 pairs), 48 log freqs 1e-3..100; "
                   "RK4 step + chi + chi(k) on 16^3 k-points", lambda: kgrid3(16)),
    "square_j1j2": ("square-lattice J1-J2 Heisenberg, J2/J1=0.5, range 7 (20 pairs), 32 log freqs "
                    "1e-3..100; RK4 step + chi + chi(k) on 64x64", lambda: kgrid(64)),
}


def hot_path_leg(name: str, steps: int, warmup: int, breakdown: bool = True) -> dict:
    """One workload's hot path on the GPU: the physical flow from the initial
    condition down to Lambda = 1 (untimed setup), then `steps` timed passes of
    [RK4 step Lambda -> 0.95 Lambda (4 self-energy + 4 vertex right-hand sides
    and the stage combinations), chi per pair, chi(k)] with HIP events on the
    vertex launches (s, u and t channels in one launch) for the roofline;
    optionally a second pass over the same steps with the channels as three
    launches and events around every kernel, for the per-kernel breakdown."""
    import torch
    from paper_2109_13317_amd import build_tables
    from paper_2109_13317_amd.flow import Context
    desc, kfun = HOT_PATH[name]
    wl = W.workload(name)
    model = wl.model()
    tables = build_tables(model, wl.range)
    ctx = Context(tables, wl.mesh)
    nf, ns = ctx.nf, ctx.ns
    E = 2 * ns * nf * nf * (nf + 1) // 2
    kp = torch.from_numpy(kfun()).cuda()
    log(f"{name}: context ready, {ns} pairs, {nf} frequencies, {E} vertex elements")
    x = ctx.init_state()
    ctx.flow(x, schedule=W.geometric_schedule(100.0, 1.0, 40), scheme="rk4")
    torch.cuda.synchronize()
    x_start = x.cpu().numpy()
    log(f"{name}: setup flow to Lambda=1 done")
    lam = [1.0]

    def step():
        l0 = lam[0]
        l1 = l0 * 0.95
        ctx.step("rk4", l0, l1, x)
        chi = ctx.chi(l1, x)
        ctx.chi_k(chi.reshape(-1), kp)
        lam[0] = l1

    for _ in range(warmup):
        step()
    lam_timed0 = lam[0]
    x_timed0 = x.clone()
    torch.cuda.synchronize()
    # timed region.  The library runs the s, u and t channels as one launch up
    # to 20 pairs (the events are handed to that launch, which stamps its own
    # start and end on the library's stream) and beyond as s+u beside a
    # concurrent t launch (events before the fork and after the join: the
    # span of the whole vertex right-hand side)
    concurrent = ns > 20
    timed = "vertex" if concurrent else "vertex_stu"
    ctx.set_profiling(True, kernels=(timed,))
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tms_t, tcount = ctx.profile_read(timed)
    ctx.set_profiling(False)
    ms_step = (t1 - t0) * 1e3 / steps
    fl = {"s": 0.0, "u": 0.0, "t": 0.0, "all": 0.0}
    l0 = lam_timed0
    for _ in range(steps):
        l1 = l0 * 0.95
        h = l1 - l0
        for ls in (l0, l0 + 0.5 * h, l0 + 0.5 * h, l1):
            f = vertex_flops(wl.mesh, ls, ns, tables.n_terms)
            for k in fl:
                fl[k] += f[k]
        l0 = l1
    tavg_ms = tms_t / max(tcount, 1)
    achieved = fl["all"] / tcount / (tavg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                "traffic": MEASURED_TRAFFIC.get((kernel_source_hash(), name)), "traffic_unit": "bytes/launch",
                "kernel": (f"vertex right-hand side: k_vertex_t<{4 * ((ns + 3) // 4)}, double> on the library stream "
                           f"beside k_vertex_su<0>, k_vertex_su<2> on its second stream, then the t-part sum "
                           "(timed from before the fork to after the join)") if concurrent else
                          f"k_vertex_stu<{4 * ((ns + 3) // 4)}, double> (s, u and t channels in one launch)",
                "launch_form": "concurrent" if concurrent else "one_launch",
                "avg_launch_ms": tavg_ms, "launches": tcount,
                "flops_per_launch": fl["all"] / tcount,
                "flops_per_launch_by_channel": {k: fl[k] / tcount for k in ("s", "u", "t")},
                "hbm_bytes_algorithmic_per_launch": 16.0 * E / 2 + 8.0 * E}
    # each launch form of the whole vertex right-hand side on the same state
    # and cutoff (the same bits), timed from before its first to after its
    # last launch
    forms = {}
    out = ctx.new_state()
    xs = torch.from_numpy(x_start).cuda()
    for form in ("one_launch", "separate", "concurrent"):
        ctx.set_vertex_mode(form)
        ctx.rhs(0.5, xs, out)
        ctx.set_profiling(True, kernels=("vertex",))
        for _ in range(5):
            ctx.rhs(0.5, xs, out)
        ms, n = ctx.profile_read("vertex")
        ctx.set_profiling(False)
        forms[form] = ms / n
    ctx.set_vertex_mode("auto")
    roofline["launch_forms_ms_at_lambda_0.5"] = forms
    log(f"{name}: vertex right-hand side at Lambda=0.5 by launch form: " +
        ", ".join(f"{k} {v:.4f} ms" for k, v in forms.items()))
    stage_lams = []
    l0 = lam_timed0
    for _ in range(steps):
        l1 = l0 * 0.95
        stage_lams += [l0, l0 + 0.5 * (l1 - l0), l1]
        l0 = l1
    res = {"workload": desc, "pairs": ns, "n_freq": nf, "vertex_elements": E, "ms_per_step": ms_step,
           "stage_lambdas": stage_lams[::max(1, len(stage_lams) // 6)],
           "value": 4 * E / (ms_step * 1e-3), "roofline": roofline, "lambda_timed": [lam_timed0, lam[0]],
           "tables": tables, "model": model, "wl": wl, "x_start": x_start, "ctx": ctx}
    log(f"{name}: {steps} steps {ms_step:.3f} ms/step, vertex launch {tavg_ms:.4f} ms, "
        f"{achieved:.2f} TFLOP/s ({roofline['frac']:.3f} of FP64 peak)")
    if breakdown:
        lam[0] = lam_timed0
        x.copy_(x_timed0)
        ctx.set_profiling(True)
        t2 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        vms, vcount = ctx.profile_read("vertex")
        parts = {k: ctx.profile_read(k)[0] for k in ("vertex_s", "vertex_u", "vertex_t", "sigma", "tables")}
        ctx.set_profiling(False)
        roofline["whole_vertex_rhs"] = {
            "avg_ms": vms / max(vcount, 1),
            "achieved_tflops": fl["all"] / vcount / (vms / vcount * 1e-3) / 1e12,
            "s_ms": parts["vertex_s"] / max(vcount, 1), "u_ms": parts["vertex_u"] / max(vcount, 1),
            "t_ms": parts["vertex_t"] / max(vcount, 1),
            "source": "a second pass over the same steps with the channels as three separate launches "
                      "(same results bitwise) and HIP events around every kernel"}
        res["kernel_ms_per_step"] = {"vertex": vms / steps, "sigma": parts["sigma"] / steps,
                                     "tables": parts["tables"] / steps,
                                     "breakdown_pass_ms_per_step": (t3 - t2) * 1e3 / steps}
    return res


def _public(d: dict) -> dict:
    return {k: v for k, v in d.items() if k not in ("tables", "model", "wl", "x_start", "ctx", "stage_lambdas")}


def adaptive_flow(ctx, kp, lam_max_breakdown, label):
    """The adaptive Dormand-Prince flow 100 -> 0.01 with chi(k) every accepted
    step (timed), then the same flow untimed recording chi_max(Lambda) for the
    breakdown detector."""
    import torch
    xf = ctx.init_state()
    torch.cuda.synchronize()
    nacc = [0]

    def obs(lam_, chi_, ck_):
        nacc[0] += 1
        if nacc[0] % 20 == 0:
            log(f"{label} adaptive flow: {nacc[0]} accepted steps, Lambda={lam_:.4g}")
        return 0

    t0 = time.perf_counter()
    nsteps = ctx.flow(xf, scheme="dopri54", lam_start=100.0, lam_stop=0.01, rtol=1e-4,
                      atol=1e-6, h0=0.05, hmin=1e-9, max_steps=20000, kpoints=kp, observer=obs)
    torch.cuda.synchronize()
    flow_s = time.perf_counter() - t0
    from paper_2109_13317_amd.breakdown import ChiMaxRecorder
    rec = ChiMaxRecorder()
    ctx.flow(ctx.init_state(), scheme="dopri54", lam_start=100.0, lam_stop=0.01, rtol=1e-4, atol=1e-6,
             h0=0.05, hmin=1e-9, max_steps=20000, kpoints=kp, observer=rec)
    chimax = np.asarray(rec.chi_max)
    bd = rec.breakdown(lam_max=lam_max_breakdown)
    log(f"{label}: adaptive flow {flow_s:.3f} s, {nsteps} steps; breakdown detector: {bd.kind} (Lambda = {bd.lam})")
    return xf, {"scheme": "dopri54 in ln Lambda, rtol 1e-4, atol 1e-6, steps land on w_n/2",
                "lambda": [100.0, 0.01], "seconds": flow_s, "accepted_steps": nsteps,
                "breakdown": {"kind": bd.kind, "lambda": bd.lam, "step": bd.index,
                              "chi_max_first": float(chimax[0]), "chi_max_last": float(chimax[-1]),
                              "detector": "first step below a quarter of the top mesh frequency with ln chi_max "
                                          "slope in ln Lambda below -8 or a slope change above 1 (heuristic, "
                                          "parity unpinned)"}}


def fixed_flow(ctx, sched):
    """The fixed RK4 flow along sched with chi at the end (timed)."""
    import torch
    from paper_2109_13317_amd._lib import PffrgError
    xf = ctx.init_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        ctx.flow(xf, schedule=sched, scheme="rk4")
        chi0 = float(ctx.chi(sched[-1], xf).reshape(-1)[0].cpu())
    except PffrgError as e:              # a flow that leaves the finite range stops there
        chi0 = f"flow stopped: {e}"
    torch.cuda.synchronize()
    return {"seconds": time.perf_counter() - t0, "steps": len(sched) - 1, "chi_zz_onsite_final": chi0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=sorted(HOT_PATH), default="pyrochlore",
                    help="the headline workload (default: pyrochlore, the largest FP64 configuration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-flow", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the second hot-path workload and the FP32, batched-scan, adjoint and scaling "
                         "measurements")
    ap.add_argument("--no-breakdown", action="store_true", help="skip the per-kernel breakdown pass")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the flow engine runs on a single MI355X "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    head = hot_path_leg(args.workload, args.steps, args.warmup, breakdown=not args.no_breakdown)
    roofline = head["roofline"]
    # the device's own peaks (FMA throughput, copy bandwidth) beside the vendor figures
    from paper_2109_13317_amd.flow import measure_peaks
    peaks = measure_peaks()
    roofline["measured_peak"] = peaks["fp64_fma_tflops"]
    roofline["frac_of_measured_peak"] = roofline["achieved"] / peaks["fp64_fma_tflops"]
    # the on-chip ceiling: every interpolation corner is one 1 KB wave gather
    # served by L1 at the measured rate
    wl_h = head["wl"]
    gi = np.mean([gather_instructions(wl_h.mesh, l, head["pairs"]) for l in head["stage_lambdas"]])
    bound_ms = gi * 1024.0 / (peaks["l1_load_tbs"] * 1e12) * 1e3
    roofline["l1_gather_bound"] = {
        "gather_instructions_per_launch": gi, "bytes_per_instruction": 1024,
        "measured_l1_tbs": peaks["l1_load_tbs"], "bound_ms": bound_ms,
        "fraction_of_bound_achieved": bound_ms / roofline["avg_launch_ms"],
        "fp64_fraction_at_bound": roofline["frac"] * roofline["avg_launch_ms"] / bound_ms}
    log(f"L1 gather bound: {gi:.3e} wave gathers per launch, {bound_ms:.4f} ms at {peaks['l1_load_tbs']:.1f} TB/s "
        f"({bound_ms / roofline['avg_launch_ms']:.2f} of the launch time)")
    log(f"measured peaks: FP64 FMA {peaks['fp64_fma_tflops']:.1f} TFLOP/s, FP32 FMA "
        f"{peaks['fp32_fma_tflops']:.1f} TFLOP/s, copy {peaks['hbm_copy_gbs']:.0f} GB/s, 16-byte lane loads: "
        f"L1 {peaks['l1_load_tbs']:.1f} TB/s (two rows {peaks['l1_load_2row_tbs']:.1f}), "
        f"LDS {peaks['lds_read_tbs']:.1f} TB/s")

    out = {
        "metric": "vertex-RHS elements/s + full-flow time vs plain FP64 GPU; adjoint/forward cost",
        "value": head["value"],
        "unit": "vertex-RHS elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": HOT_PATH[args.workload][0], "pairs": head["pairs"], "n_freq": head["n_freq"],
                   "vertex_elements": head["vertex_elements"], "parallelism": "single GPU",
                   "lambda_timed": head["lambda_timed"]},
        "roofline": roofline,
        "measured_peaks": {**peaks, "method": "pffrg_measure_peaks: 8 FMA chains per lane on every CU "
                                              "(FP32 without packed instructions); 512 MiB device copy; "
                                              "128-bit lane loads from a 16 KB L1-resident buffer and from LDS"},
    }
    if "kernel_ms_per_step" in head:
        out["kernel_ms_per_step"] = head["kernel_ms_per_step"]

    if not args.no_full_flow:
        ctx, wl = head["ctx"], head["wl"]
        kp = torch.from_numpy(HOT_PATH[args.workload][1]()).cuda()
        flows = {}
        if wl.schedule is not None:
            log(f"{args.workload}: fixed RK4 flow")
            flows["fixed_rk4"] = {"schedule": "exponential Lambda_n = 100 * 0.95^n down to 0.01",
                                  **fixed_flow(ctx, list(wl.schedule))}
        xf, flows["adaptive"] = adaptive_flow(ctx, kp, wl.mesh[-1] / 4, args.workload)
        flows["adaptive"]["chi_k_every_step"] = f"{len(kp)} k-points"
        flows["checkpoint"] = checkpoint_cost(xf)
        out["full_flow"] = flows

    if not args.no_extras:
        other = "square_j1j2" if args.workload == "pyrochlore" else "pyrochlore"
        sec = hot_path_leg(other, args.steps, args.warmup, breakdown=False)
        out[other] = _public(sec)
        if not args.no_full_flow and other == "square_j1j2":
            kp2 = torch.from_numpy(HOT_PATH[other][1]()).cuda()
            _, out[other]["full_flow"] = adaptive_flow(sec["ctx"], kp2, sec["wl"].mesh[-1] / 4, other)
        sq = head if args.workload == "square_j1j2" else sec
        log("FP32 mode")
        out["fp32_mode"] = fp32_leg(sq["tables"], sq["wl"], sq["x_start"], 0.5)
        log("batched scan")
        out["batch_scan"] = batch_leg()
        log("adjoint")
        out["adjoint"] = adjoint_leg()
        log("XYZ")
        out["xyz"] = xyz_leg()
        log("TRI")
        out["tri"] = tri_leg()
        log("scaling shape")
        out["scaling_shape"] = scaling_leg()
    out["paper_context"] = {
        "value": 2.6e6, "unit": "vertex elements per second per node",
        "hardware": "Intel Xeon Phi 7250-F node (68 cores, 1.4 GHz)",
        "workload": "cubic J1-J2, range 7 (31 pairs), 64 frequencies, Euler steps with correlations",
        "derivation": "about 25 core-hours for 422 steps of 8.25 M vertex elements, perfect scaling assumed"}

    if args.copy_probe:
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = a.numel() * 8

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        out["cpu_baseline"] = cpu_baseline(head["model"], head["wl"], head["tables"], head["x_start"], 1.0)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
