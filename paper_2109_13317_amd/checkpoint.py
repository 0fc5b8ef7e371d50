"""Flow checkpoints: full snapshots of a running flow, written at a time
interval, from which an interrupted flow resumes exactly and a finished one
extends to lower cutoffs (the checkpoint files of Sec. 5 and 5.1 of
arXiv:2109.13317: a snapshot of the whole calculation, a status of running or
finished, start, checkpoint and end times).

A snapshot holds the flow state and a JSON record: the calculation's identity
(mesh, a digest of the lattice tables, precision, scheme with its tolerances
or schedule), the position of the last accepted step as the integrator holds
it (``Context.position``: ln Lambda and the adaptive controller's step index,
or the schedule index) and the status.  Resuming hands that position back to
the library, so the resumed flow takes bitwise the steps the uninterrupted
one would have taken.  Files are NumPy ``.npz`` archives (no pickled objects)
written to a temporary name and renamed, so an interrupted write leaves the
previous snapshot intact.
"""

from __future__ import annotations

import datetime
import hashlib
import json
import os
import time
from dataclasses import dataclass

import numpy as np

from . import _lib

FORMAT = 1


def _hex(v) -> str:
    return float(v).hex()


def _unhex(s: str) -> float:
    return float.fromhex(s)


def _now() -> str:
    return datetime.datetime.now().isoformat(timespec="seconds")


def lattice_digest(tables) -> str:
    """SHA-256 over the lattice tables the flow depends on."""
    h = hashlib.sha256()
    h.update(np.int64(tables.n_pairs).tobytes())
    for a, dt in ((tables.swap, np.int32), (tables.mult, np.int32), (tables.rpa_off, np.int32),
                  (tables.rpa_ka, np.int32), (tables.rpa_kb, np.int32), (tables.rpa_cnt, np.int32),
                  (tables.coupling, np.float64)):
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    return h.hexdigest()


@dataclass
class Snapshot:
    state: np.ndarray     # float64, the context's state layout
    meta: dict


def write(path: str, state: np.ndarray, meta: dict) -> None:
    """Write a snapshot atomically (temporary file, fsync, rename)."""
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, state=np.ascontiguousarray(state, dtype=np.float64),
                 meta=np.array(json.dumps(meta, sort_keys=True)))
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)


def read(path: str) -> Snapshot:
    with np.load(path, allow_pickle=False) as z:
        state = np.array(z["state"], dtype=np.float64)
        meta = json.loads(str(z["meta"]))
    if meta.get("format") != FORMAT:
        raise ValueError(f"{path}: unknown checkpoint format {meta.get('format')!r}")
    return Snapshot(state, meta)


def identity(ctx, scheme: str, *, schedule=None, rtol=None, atol=None, h0=None, hmin=None) -> dict:
    """What must match for a snapshot to continue a flow (the adaptive
    flow's lam_stop and a fixed schedule's tail may change: they extend it)."""
    ident = {"format": FORMAT, "mesh": [_hex(w) for w in ctx.mesh], "lattice": lattice_digest(ctx.tables),
             "precision": ctx.precision, "size": int(ctx.size), "scheme": scheme}
    if scheme == "dopri54":
        ident.update(rtol=_hex(rtol), atol=_hex(atol), h0=_hex(h0), hmin=_hex(hmin))
    else:
        ident["schedule"] = [_hex(v) for v in schedule]
    return ident


def _check_identity(saved: dict, ident: dict, path: str) -> None:
    for k, v in ident.items():
        if k == "schedule":
            old = saved.get("schedule", [])
            if v[:len(old)] != old:
                raise ValueError(f"{path}: the schedule does not continue the checkpointed one")
        elif saved.get(k) != v:
            raise ValueError(f"{path}: checkpoint belongs to another calculation ({k} differs)")


def flow(ctx, x, path: str, *, scheme: str = "rk4", schedule=None, lam_start=None, lam_stop=None,
         rtol=1e-6, atol=1e-10, h0=0.05, hmin=1e-8, max_steps=0, kpoints=None, observer=None,
         every: float = 3600.0, force_restart: bool = False) -> int:
    """``Context.flow`` with checkpoints in ``path``, written after the first
    accepted step at least ``every`` seconds after the previous snapshot, and
    at the end.  If ``path`` holds a snapshot of the same calculation and
    ``force_restart`` is false, the flow continues from it: an interrupted
    flow resumes where it stopped, a finished one extends to a lower lam_stop
    (adaptive) or a longer schedule (fixed); ``x`` receives the snapshot's
    state.  Returns the accepted steps of this call.  A flow that diverges
    leaves a snapshot with status "diverged" and raises."""
    import torch

    if scheme not in ("euler", "rk4", "dopri54"):
        raise ValueError(f"unknown scheme {scheme!r}")
    sched = None if scheme == "dopri54" else [float(v) for v in schedule]
    ident = identity(ctx, scheme, schedule=sched, rtol=rtol, atol=atol, h0=h0, hmin=hmin)
    meta = dict(ident, status="running", start_time=_now(), steps=0)
    resume = None
    offset = 0            # fixed schedules: index of the flow's first cutoff
    if not force_restart and os.path.exists(path):
        snap = read(path)
        _check_identity(snap.meta, ident, path)
        if snap.meta["status"] == "diverged":
            raise _lib.PffrgError(_lib.EDIVERGED, f"{path}: the checkpointed flow diverged "
                                                  f"(restart with force_restart=True)")
        if snap.state.size != ctx.size:
            raise ValueError(f"{path}: state size differs")
        x.copy_(torch.from_numpy(snap.state))
        meta.update(start_time=snap.meta["start_time"], steps=snap.meta["steps"])
        if scheme == "dopri54":
            lend = float(np.log(lam_stop))
            if not _unhex(snap.meta["log_lambda"]) > lend:
                return 0
            resume = (_unhex(snap.meta["log_lambda"]), int(snap.meta["ladder"]))
        else:
            offset = int(snap.meta["ladder"])
            if offset >= len(sched) - 1:
                return 0
    run_sched = None if sched is None else sched[offset:]
    last = [time.monotonic()]

    def save(status: str) -> None:
        lam, ll, lad = ctx.position()
        meta.update(status=status, checkpoint_time=_now(), **{"lambda": _hex(lam)}, log_lambda=_hex(ll),
                    ladder=int(lad) + offset)
        if status != "running":
            meta["end_time"] = meta["checkpoint_time"]
        if sched is not None:
            meta["schedule"] = [_hex(v) for v in sched[:offset + lad + 1]]
            meta["lambda_stop"] = _hex(sched[-1])
        else:
            meta["lambda_stop"] = _hex(lam_stop)
        torch.cuda.current_stream().synchronize()
        write(path, x.detach().cpu().numpy(), meta)
        last[0] = time.monotonic()

    def obs(lam, chi, chik):
        stop = bool(observer(lam, chi, chik)) if observer is not None else False
        meta["steps"] += 1
        if time.monotonic() - last[0] >= every:
            save("running")
        return stop

    try:
        n = ctx.flow(x, schedule=run_sched, scheme=scheme, lam_start=lam_start, lam_stop=lam_stop, rtol=rtol,
                     atol=atol, h0=h0, hmin=hmin, max_steps=max_steps, kpoints=kpoints, observer=obs,
                     resume=resume)
    except _lib.PffrgError as e:
        if e.status == _lib.EDIVERGED and meta["steps"] > 0:
            save("diverged")
        raise
    if n > 0:
        lam, ll, lad = ctx.position()
        done = (lad + offset >= len(sched) - 1) if sched is not None else not (ll > float(np.log(lam_stop)))
        save("finished" if done else "running")
    return n


def batch_identity(batch, schedule) -> dict:
    """What must match for a snapshot to continue a batch flow (the schedule
    may be extended)."""
    return {"format": FORMAT, "kind": "batch", "mesh": [_hex(w) for w in batch.mesh],
            "lattices": [lattice_digest(t) for t in batch.tables], "precision": batch.precision,
            "size": int(batch.size), "scheme": "rk4", "schedule": [_hex(v) for v in schedule]}


def batch_flow(batch, x, path: str, schedule, *, every: float = 3600.0, segment: int = 8,
               force_restart: bool = False, use_graph: bool = True) -> list[bool]:
    """``Batch.flow`` with checkpoints in ``path``.  The schedule runs in
    segments of ``segment`` RK4 steps (one batch launch sequence each; the
    steps are those of one call over the whole schedule, so the states are
    bitwise the same); after a segment ending at least ``every`` seconds after
    the previous snapshot, and at the end, the batch state is written with
    the schedule index reached and each point's finiteness.  A snapshot of
    the same batch (points, mesh, precision, a schedule that the given one
    continues) is resumed from unless ``force_restart``.  Returns each
    point's finiteness at the end."""
    import torch

    sched = [float(v) for v in schedule]
    if len(sched) < 2 or segment < 1:
        raise ValueError("a batch flow needs >= 2 cutoffs and segment >= 1")
    ident = batch_identity(batch, sched)
    meta = dict(ident, status="running", start_time=_now(), steps=0)
    start, ok = 0, [True] * batch.n_points
    if not force_restart and os.path.exists(path):
        snap = read(path)
        _check_identity(snap.meta, ident, path)
        if snap.state.size != batch.size:
            raise ValueError(f"{path}: state size differs")
        x.copy_(torch.from_numpy(snap.state))
        start, ok = int(snap.meta["index"]), [bool(v) for v in snap.meta["finite"]]
        meta.update(start_time=snap.meta["start_time"], steps=snap.meta["steps"])
        if start >= len(sched) - 1:
            return ok
    last = time.monotonic()

    def save(status: str, i: int) -> None:
        meta.update(status=status, checkpoint_time=_now(), index=i, finite=ok,
                    schedule=[_hex(v) for v in sched[:i + 1]], **{"lambda": _hex(sched[i])})
        if status != "running":
            meta["end_time"] = meta["checkpoint_time"]
        torch.cuda.current_stream().synchronize()
        write(path, x.detach().cpu().numpy(), meta)

    i = start
    while i < len(sched) - 1:
        j = min(i + segment, len(sched) - 1)
        seg_ok = batch.flow(x, sched[i:j + 1], use_graph=use_graph)
        ok = [a and b for a, b in zip(ok, seg_ok)]
        meta["steps"] += j - i
        i = j
        if i < len(sched) - 1 and time.monotonic() - last >= every:
            save("running", i)
            last = time.monotonic()
    save("finished", i)
    return ok

