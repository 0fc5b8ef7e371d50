"""Flow breakdown: where the cutoff dependence of the peak susceptibility
chi_max(Lambda) = max_k chi(k, Lambda) stops being smooth.

In pf-FRG a transition into a phase that breaks a symmetry of the
parametrisation shows up as a divergence or a kink of chi_max as a function of
Lambda, while symmetric (spin-liquid) phases flow smoothly (Sec. 3 of
arXiv:2109.13317, after Eq. 31); mapping phase diagrams means locating that
point.  The paper names the signatures but fixes no criterion, so this is a
heuristic on the accepted steps of a flow, in y = ln chi_max against
t = ln Lambda:

* non-finite (or non-positive) chi_max: "nonfinite";
* a local slope dy/dt below -max_slope (chi_max growing faster than
  Lambda^-max_slope, as it does approaching a pole): "divergence";
* a slope that changes by more than max_kink between consecutive steps (the
  smooth parts of a flow change it by far less per step): "kink".

The first accepted step that meets one of them is reported.  Steps above
lam_max are skipped: where the cutoff is near the top of the frequency mesh it
removes mesh frequencies and chi_max grows from almost zero, steeply and
unevenly, for reasons of the mesh alone (a quarter of the largest mesh
frequency is a safe bound on logarithmic meshes).

On square J1-J2, range 7, 32 frequencies (adaptive flow 100 -> 0.01, chi(k) on
64 x 64 points, lam_max = 25) this flags J2/J1 = 0 (Neel order) at Lambda =
0.55 and J2/J1 = 1 (stripe order) at 0.38 as kinks and finds J2/J1 = 0.5
smooth, as pf-FRG studies of this model do.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Breakdown:
    kind: str | None        # "nonfinite", "divergence", "kink", or None (smooth)
    index: int | None       # accepted step at which it was detected
    lam: float | None       # its cutoff


def find_breakdown(lams, chi_max, *, max_slope: float = 8.0, max_kink: float = 1.0,
                   lam_max: float = np.inf) -> Breakdown:
    """First breakdown along a flow (lams in the order of the flow; steps
    above lam_max are skipped)."""
    lam = np.asarray(lams, dtype=np.float64)
    chi = np.asarray(chi_max, dtype=np.float64)
    if lam.shape != chi.shape or lam.ndim != 1:
        raise ValueError("lams and chi_max must be 1-D of equal length")
    prev, prev_slope = None, None
    for i in range(len(lam)):
        if not (np.isfinite(chi[i]) and chi[i] > 0.0):
            return Breakdown("nonfinite", i, float(lam[i]))
        if lam[i] > lam_max:
            continue
        if prev is None:
            prev = i
            continue
        dt = np.log(lam[i]) - np.log(lam[prev])
        if dt == 0.0:
            continue
        slope = (np.log(chi[i]) - np.log(chi[prev])) / dt
        prev = i
        if slope < -max_slope:
            return Breakdown("divergence", i, float(lam[i]))
        if prev_slope is not None and abs(slope - prev_slope) > max_kink:
            return Breakdown("kink", i, float(lam[i]))
        prev_slope = slope
    return Breakdown(None, None, None)


class ChiMaxRecorder:
    """Observer for ``Context.flow`` (or ``checkpoint.flow``) that records the
    cutoff and chi_max of every accepted step: the maximum of chi(k) over the
    flow's k-points, or of chi^zz over the pairs when none were given."""

    def __init__(self):
        self.lams: list[float] = []
        self.chi_max: list[float] = []

    def __call__(self, lam, chi_pairs, chi_k):
        src = chi_k if chi_k is not None else chi_pairs[0]
        self.lams.append(float(lam))
        self.chi_max.append(float(src.max()))
        return False

    def breakdown(self, **kw) -> Breakdown:
        return find_breakdown(self.lams, self.chi_max, **kw)


def batch_breakdowns(batch, x, schedule, kpoints, *, use_graph: bool = True, record=None, **kw):
    """Advance a batch (``flow.Batch``) along an RK4 schedule one step at a
    time, in place, recording chi_max = max over kpoints of chi(k) for every
    point after every step, and locate each point's breakdown (keyword
    arguments as find_breakdown).  The steps are those of one
    ``Batch.flow`` call over the schedule.  If record is a list, every step
    appends (Lambda, per-point finiteness of the state, per-point chi as host
    arrays).  Returns (breakdowns, lams, chi_max[point][step])."""
    import torch
    sched = [float(v) for v in schedule]
    lams, maxima = [], []
    for i in range(len(sched) - 1):
        ok = batch.flow(x, sched[i:i + 2], use_graph=use_graph)
        chis = batch.chi(sched[i + 1], x)
        maxima.append(torch.stack([batch.chi_k(p, c, kpoints).max() for p, c in enumerate(chis)]))
        lams.append(sched[i + 1])
        if record is not None:
            record.append((sched[i + 1], ok, [c.cpu().numpy() for c in chis]))
    chi_max = torch.stack(maxima, 1).cpu().numpy()
    return [find_breakdown(lams, chi_max[p], **kw) for p in range(batch.n_points)], lams, chi_max

