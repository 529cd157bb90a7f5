"""Reference of the uncertainty-aware semantic-on-demand scheduler
(Sec. IV-B, Eq. (13)-(17)) and of a sequence of MP updates driven by it.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Per frame t: the frame uncertainty U_bar (Eq. (13), the lower median of the
normalised uncertainty over the Gaussians the last MP update observed), the
tracking inconsistency R = clip(e_bar / e_ref, 0, 1) (Eq. (14)), the score
S = w_u U_bar + w_r R (Eq. (15)), and a refresh of the instance prior when
S > theta or dt >= N_max (Eq. (16)); without a refresh the MP update runs on
the last refreshed masks with alpha' = rho alpha (Eq. (17)). Constants (the
paper names them without values): theta = 0.5, N_max = 10, w_u = w_r = 0.5,
e_ref = 2 px. Readings:
  * the decision at frame t uses the U_bar of the latest MP update (frame
    t - 1; the update of frame t needs the decision first) and the R of
    frame t;
  * e_bar is the mean of the median epipolar distances (Eq. (18)-(19)) of the
    frame's candidates that MP labels static (NOT_SUPPRESSED) with a finite
    median: the correspondences the tracker trusts; 0 when there are none;
  * dt counts the frames since the last refresh including the current one,
    and starts at N_max, so the first frame refreshes.

Pinned by tests/test_oracle_scheduler.py: hand-built sequences (the max-skip
rule alone gives refreshes every N_max frames, a score above theta refreshes
and restarts the count, theta itself does not trigger, R saturates at 1), and
the MP sequence against single frames of the MP reference with the masks and
rate the decisions imply.
"""

from __future__ import annotations

import numpy as np

from . import mp as omp

DEFAULTS = dict(w_u=0.5, w_r=0.5, theta=0.5, e_ref=2.0, n_max=10)
NOT_SUPPRESSED = 2


def e_bar_of(dbar, epi_state) -> float:
    dbar = np.asarray(dbar, dtype=np.float64)
    sel = (np.asarray(epi_state) == NOT_SUPPRESSED) & np.isfinite(dbar)
    return float(dbar[sel].mean()) if sel.any() else 0.0


class Scheduler:
    """Eq. (14)-(16) with the frame counter of the max-skip rule."""

    def __init__(self, **kw):
        self.p = dict(DEFAULTS)
        self.p.update(kw)
        self.dt = self.p["n_max"]
        self.n_refresh = 0
        self.S = self.R = self.e_bar = None

    def decide(self, U_bar, e_bar) -> bool:
        p = self.p
        self.e_bar = e_bar
        self.R = min(max(e_bar / p["e_ref"], 0.0), 1.0)
        u = 0.0 if np.isnan(U_bar) else U_bar
        self.S = p["w_u"] * u + p["w_r"] * self.R
        go = self.S > p["theta"] or self.dt >= p["n_max"]
        if go:
            self.dt = 1
            self.n_refresh += 1
        else:
            self.dt += 1
        return go


def run_mp_sequence(frames, params=None, sched=None, policy="on_demand", n_fixed=10):
    """MP updates over `frames` (dicts of one MP update's inputs, each with the
    fresh instance masks of its frame and the medians and states of its
    epipolar verification candidates) under a policy:
    'always' refreshes every frame, 'fixed' every n_fixed frames, 'on_demand'
    by the scheduler. The first frame's mp is the starting state; later
    frames take the state the previous update left. Returns per frame the
    refresh decision, the scheduler's S and the MP reference's result."""
    sch = Scheduler(**(sched or {}))
    mp = np.asarray(frames[0]["mp"], dtype=np.float32).copy()
    U_prev = 0.0
    masks = None
    out = []
    for t, fr in enumerate(frames):
        if policy == "always":
            go = True
        elif policy == "fixed":
            go = t % n_fixed == 0
        else:
            go = sch.decide(U_prev, e_bar_of(fr["dbar"], fr["epi_state"]))
        if go or masks is None:
            masks = fr["instance_id"]
        inp = dict(fr)
        inp["instance_id"] = masks
        inp["mp"] = mp
        r = omp.mp_update(inp, params, seg_updated=bool(go))
        mp = r["mp"].astype(np.float32)
        U_prev = float(r["stats"]["U_bar"])
        out.append(dict(refresh=bool(go), S=sch.S if policy == "on_demand" else None, result=r))
    return out
