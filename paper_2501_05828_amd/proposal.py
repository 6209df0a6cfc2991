"""Learned emission proposal driven through the C ABI.

record(): trace with uniform emission while the library appends every binned
contribution (row, emission cell, |c|); with cost_aware, also the cost of
every path per emission cell, after which each record is reweighted so that
the training target per cell is sqrt(sum c^2 / mean path cost) -- the
density that minimises variance x time -- instead of sum |c|.  train(): Adam
steps on minibatch histograms drawn from those records.  enable(): the network's direction
distribution, mixed with eps of uniform, becomes the emission pdf of later
traces (weights 1/pdf keep the estimator unbiased).  save()/load(): the
training state (parameters, Adam moments, step) as an .npz checkpoint.
"""
from __future__ import annotations

import torch

from . import scenes


class Proposal:
    def __init__(self, sim, seed: int = 7):
        self.sim = sim
        self.ctx = sim.ctx
        params, rff = scenes.proposal_init(seed)
        self.ctx.ur_mlp_init(params, rff)
        a = sim.w.acq
        self.rows = a.n_tx * a.n_elements
        dev = sim.dev
        self.hist = torch.zeros((self.rows, 1024), dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.pdf = torch.empty((self.rows, 1024), dtype=torch.float32, device=dev)
        self.cdf = torch.empty((self.rows, 1024), dtype=torch.float32, device=dev)
        self.rec = None
        self.n_rec = 0

    def record(self, n_traces: int, cap: int = 1 << 22, seed0: int = 0x1234_0000, cost_aware: bool = False):
        """Records contributions of n_traces uniform traces of the current
        acquisition; returns (records kept, records offered)."""
        dev = self.sim.dev
        self.rec = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        cost = torch.zeros((self.rows, 1024), dtype=torch.float32, device=dev) if cost_aware else None
        self.ctx.ur_set_proposal(None, None)
        self.ctx.ur_set_record(self.rec, count)
        if cost_aware:
            self.ctx.ur_set_cost_histogram(cost)
        try:
            for i in range(n_traces):
                self.sim.trace(seed=seed0 + i, pulse=False)
        finally:
            self.ctx.ur_set_record(None)
            self.ctx.ur_set_cost_histogram(None)
        offered = int(count.item())
        self.n_rec = min(offered, cap)
        if cost_aware and self.n_rec:
            rays_per_row = float(self.sim.w.acq.rays_per_element) * n_traces
            self.ctx.ur_record_reweight(self.rec, self.n_rec, cost, rays_per_row)
        self.cost = cost
        return self.n_rec, offered

    def train(self, steps: int = 2000, batch: int = 1 << 16, lr: float = 1e-3, seed: int = 11,
              log_every: int = 0):
        if self.n_rec == 0:
            raise RuntimeError("no recorded contributions to train on")
        losses = []
        for step in range(steps):
            self.ctx.ur_record_histogram(self.rec, self.n_rec, batch, seed, step, self.hist)
            self.ctx.ur_mlp_train_step(self.hist, lr, self.loss)
            if log_every and (step % log_every == 0 or step == steps - 1):
                losses.append((step, float(self.loss.item())))
        return losses

    def save(self, path: str):
        """Writes the training state (parameters, Adam moments, step) to an
        .npz file."""
        import numpy as np
        state, step = self.ctx.ur_mlp_get_state()
        np.savez(path, state=state, step=np.int64(step))

    def load(self, path: str):
        """Restores a state written by save() for the same transmit setup."""
        import numpy as np
        with np.load(path) as f:
            self.ctx.ur_mlp_set_state(f["state"], int(f["step"]))

    def enable(self, eps: float = 0.1):
        self.ctx.ur_mlp_proposal_tables(eps, self.pdf, self.cdf)
        self.ctx.ur_set_proposal(self.pdf, self.cdf)

    def disable(self):
        self.ctx.ur_set_proposal(None, None)
