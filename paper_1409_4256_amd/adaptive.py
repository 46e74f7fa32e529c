"""Adaptive EMC (Section 3.4): EMC iterations on the 600-cell rotation set of
refinement d (eq. (2.7)), with d raised by one whenever the mean log-evidence
changed by at most `tol` of its value since the previous iteration (eq. (3.1)),
up to d_max.  Early iterations run on coarse, cheap rotation sets; the fine sets
are used once the coarse ones stop improving the likelihood.

Every iteration is one `emc_iterate` call of the C ABI; the packed frames do not
depend on the rotation set and are packed once, while the geometry, its
brick-major c-step plan and the workspace are rebuilt when d changes.
"""
from __future__ import annotations

import time

from . import emc
from .rotations import next_refinement, rotation_set


class AdaptiveEMC:
    def __init__(self, grid_n, q, mask, counts_dev, d_start, d_max, precision=emc.EMC_PREC_BF16, tol=0.01,
                 brick=True):
        import torch

        if not 1 <= d_start <= d_max:
            raise ValueError("need 1 <= d_start <= d_max")
        self.grid_n, self.q, self.mask = grid_n, q, mask
        self.n_data = int(counts_dev.shape[0])
        self.precision, self.tol, self.brick = precision, tol, brick
        self.d, self.d_max = d_start, d_max
        self._build(d_start)
        self.K = emc.frames_tensor(self.geo)
        emc.emc_pack_frames(self.geo, counts_dev, self.K)
        self.loglik = torch.empty(1, dtype=torch.float64, device="cuda")
        self.L_prev = None
        self.history = []   # (iteration, d, n_rot, mean log-evidence, GPU ms, wall ms incl. any rebuild)

    def _build(self, d):
        import torch

        quat, log_w = rotation_set(d)
        self.geo = emc.Geometry(self.grid_n, torch.as_tensor(self.q), torch.as_tensor(self.mask),
                                torch.as_tensor(quat), torch.as_tensor(log_w), self.n_data, self.precision)
        if self.brick:
            self.geo.use_brick_scatter()
        self.ws = torch.empty(emc.emc_workspace_bytes(self.geo), dtype=torch.uint8, device="cuda")

    def step(self, model_in, model_out):
        """One EMC iteration at the current d, then the refinement rule."""
        import torch

        t0 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        emc.emc_iterate(self.geo, model_in, self.K, model_out, self.loglik, ws=self.ws)
        e1.record()
        torch.cuda.synchronize()
        L = self.loglik.item()
        rec = [len(self.history) + 1, self.d, self.geo.n_rot, L, e0.elapsed_time(e1)]
        d_next = next_refinement(self.L_prev, L, self.d, self.d_max, self.tol)
        self.L_prev = L
        if d_next != self.d:
            self.d = d_next
            self._build(d_next)
            torch.cuda.synchronize()
        self.history.append(tuple(rec + [(time.perf_counter() - t0) * 1e3]))
        return L

    def run(self, model, n_iter):
        """n_iter iterations from `model` (float tensor [N^3] on the GPU); returns the final model."""
        import torch

        cur, nxt = model.clone(), torch.empty_like(model)
        t0 = time.perf_counter()
        for _ in range(n_iter):
            self.step(cur, nxt)
            cur, nxt = nxt, cur
        self.wall_s = time.perf_counter() - t0
        return cur
