"""Semantic-on-demand scheduling of the instance prior (Sec. IV-B, Eq.
(13)-(17)) over a sequence of MP updates.

Each frame: decide whether to refresh the instance prior (gs_sched_decide,
from the frame uncertainty U_bar of the latest gs_mp_update and the frame's
epipolar candidates), then run gs_mp_update on the refreshed masks with
seg_updated = 1, or on the last refreshed masks with seg_updated = 0 (the
rate alpha' = rho alpha of Eq. (17)). Policies: 'on_demand' (the scheduler),
'always' (every frame) and 'fixed' (every n_fixed frames), the three rows of
the scheduling ablation. The decision at frame t uses the U_bar of frame
t - 1, since the update of frame t needs the decision first.
"""

from __future__ import annotations

import torch

from . import gs


class PriorScheduler:
    """Holds the instance masks the MP update uses and the scheduler state."""

    def __init__(self, n_pixels, policy="on_demand", n_fixed=10, device="cuda", **sched):
        if policy not in ("on_demand", "always", "fixed"):
            raise ValueError(f"unknown policy {policy!r}")
        self.policy, self.n_fixed = policy, int(n_fixed)
        self.params = gs.sched_params(**sched)
        self.state = gs.sched_state(self.params)
        self.masks = torch.zeros(n_pixels, dtype=torch.int32, device=device)
        self.have = False
        self.t = 0
        self.U_prev = 0.0
        self.refreshes = 0
        self.last = False

    def decide(self, dbar=None, epi_state=None) -> bool:
        """Whether frame t refreshes the prior. dbar, epi_state: the frame's
        epipolar candidates on the host (numpy), used by 'on_demand'."""
        if self.policy == "always":
            go = True
        elif self.policy == "fixed":
            go = self.t % self.n_fixed == 0
        else:
            go = gs.gs_sched_decide(self.params, self.state, self.U_prev, dbar, epi_state)
        go = go or not self.have
        self.refreshes += int(go)
        self.last = go
        return go

    def prior(self, fresh_masks):
        """The masks this frame's MP update uses: the fresh ones (copied) when
        the prior is refreshed, the last refreshed ones otherwise."""
        if self.last:
            self.masks.copy_(fresh_masks)
            self.have = True
        return self.masks

    def observe(self, stats):
        """After the frame's gs_mp_update: keep its U_bar (stats[0], a device
        read) for the next decision."""
        self.U_prev = float(stats[0])
        self.t += 1
