"""Driver of the learned orientation proposal (control flow over the C ABI only).

Every computation runs in libemc.so: network preprocessing, forward, gradients,
Adam, top-K, training targets, the proposal plan and the restricted iteration.
This module sequences those calls: it collects training targets from full
iterations, trains the network on them, builds the plan, and runs restricted
iterations with the recall audit deciding the fallback to the full search.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import emc as E

RECALL_MIN = 0.98


def init_params(rng: np.random.Generator, n_cells: int) -> torch.Tensor:
    """He-normal weights, zero biases, in the library's parameter layout (random numbers
    drawn on the host and handed to the device, like every other input)."""
    chans = (1, 32, 64, 128, 128)
    parts = []
    for l in range(4):
        ci, co = chans[l], chans[l + 1]
        parts.append(rng.standard_normal(co * ci * 9) * math.sqrt(2.0 / (ci * 9)))
        parts.append(np.zeros(co))
    parts.append(rng.standard_normal(n_cells * 2048) * math.sqrt(2.0 / 2048))
    parts.append(np.zeros(n_cells))
    v = np.concatenate(parts).astype(np.float32)
    assert v.size == E.emc_cnn_param_count(n_cells)
    return torch.as_tensor(v, device="cuda")


class CellIndex:
    """Fine rotations grouped by coarse cell (CSR), computed by the library's plan kernels."""

    def __init__(self, geo: E.Geometry, coarse: torch.Tensor, n_cells: int):
        # a plan over a single empty frame gives the rotation grouping
        one = geo.with_frames(1)
        topk = torch.zeros(1, dtype=torch.int32, device="cuda")
        counts = torch.zeros(geo.n_pix, dtype=torch.uint16, device="cuda")
        self.buf = torch.empty(E.emc_proposal_bytes(one, n_cells, 1, 0, 1), dtype=torch.uint8, device="cuda")
        plan = E.emc_proposal_build(one, coarse, n_cells, topk, 1, None, counts, 1, self.buf)
        self.cell_of = E.plan_array(self.buf, plan.cell_of, geo.n_rot, torch.int32).clone()
        ptr64 = E.plan_array(self.buf, plan.cell_ptr, n_cells + 1, torch.int64)
        self.cell_ptr = ptr64.to(torch.int32).clone()
        self.cell_rot = E.plan_array(self.buf, plan.cell_rot, geo.n_rot, torch.int32).clone()
        del self.buf


@dataclasses.dataclass
class TrainLog:
    steps: int
    epochs: int
    loss_first: float
    loss_last: float
    seconds: float


class Network:
    def __init__(self, n_cells: int, params: torch.Tensor, batch: int = 256):
        self.n_cells = n_cells
        self.params = params
        self.batch = batch
        self.ws = torch.empty(E.emc_cnn_workspace_bytes(n_cells, batch), dtype=torch.uint8, device="cuda")
        n = E.emc_cnn_param_count(n_cells)
        self.grads = torch.zeros(n, dtype=torch.float32, device="cuda")
        self.m = torch.zeros_like(self.grads)
        self.v = torch.zeros_like(self.grads)
        self.step = 0

    def images(self, geo: E.Geometry, K, bins: torch.Tensor) -> torch.Tensor:
        x = torch.empty(geo.n_data * 4096, dtype=torch.float32, device="cuda")
        E.emc_cnn_preprocess(geo, K, bins, None, geo.n_data, x)
        return x

    def train(self, x: torch.Tensor, targets: list, frames_per_set: int, epochs: int, lr: float,
              rng: np.random.Generator) -> TrainLog:
        """Adam on minibatches of (frame image, cell target) pairs drawn from every target
        set (the minibatches are gathered on the device; nothing waits for the GPU
        between steps)."""
        import time

        B, nc = self.batch, self.n_cells
        n_sets = len(targets)
        total = n_sets * frames_per_set
        T_all = torch.cat([t.view(-1, nc) for t in targets])      # [set * frames + frame][cell]
        xb = torch.empty(B, 4096, dtype=torch.float32, device="cuda")
        tb = torch.empty(B, nc, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        first = last = float("nan")
        t0 = time.perf_counter()
        steps = 0
        x2 = x.view(-1, 4096)
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(total), device="cuda")
            for s in range(0, total - B + 1, B):
                idx = perm[s:s + B]
                torch.index_select(x2, 0, idx % frames_per_set, out=xb)
                torch.index_select(T_all, 0, idx, out=tb)
                E.emc_cnn_gradients(nc, self.params, xb, tb, B, self.grads, loss, self.ws)
                self.step += 1
                E.emc_cnn_adam(nc, self.params, self.grads, self.m, self.v, self.step, lr)
                steps += 1
                if steps == 1:
                    first = loss.item()
        last = loss.item()
        torch.cuda.synchronize()
        del T_all
        return TrainLog(steps, epochs, first, last, time.perf_counter() - t0)

    def topk(self, x: torch.Tensor, n_frames: int, k: int) -> torch.Tensor:
        B, nc = self.batch, self.n_cells
        logits = torch.empty(B * nc, dtype=torch.float32, device="cuda")
        out = torch.empty(n_frames * k, dtype=torch.int32, device="cuda")
        x2 = x.view(-1, 4096)
        for s in range(0, n_frames, B):
            nb = min(B, n_frames - s)
            E.emc_cnn_forward(nc, self.params, x2[s:s + nb].reshape(-1), nb, logits, self.ws)
            E.emc_cnn_topk(logits, nb, nc, k, out[s * k:(s + nb) * k])
        return out


class ProposedIteration:
    """Plan + packed audited frames + workspace for emc_iterate_proposed."""

    def __init__(self, geo16: E.Geometry, counts_dev, coarse, n_cells, topk, k_top, audit, nz_cap=None):
        self.geo = geo16
        if nz_cap is None:  # non-zero pixels of all frames (an upper bound of the candidate frames')
            nz_cap = int((counts_dev.view(torch.int16) != 0).sum().item())
        n_audit = 0 if audit is None else audit.numel()
        self.buf = torch.empty(E.emc_proposal_bytes(geo16, n_cells, k_top, n_audit, max(1, nz_cap)),
                               dtype=torch.uint8, device="cuda")
        self.plan = E.emc_proposal_build(geo16, coarse, n_cells, topk, k_top, audit, counts_dev, max(1, nz_cap),
                                         self.buf)
        p = self.plan
        self.cand_frames = E.plan_array(self.buf, p.cand_frames, p.n_cand, torch.int32)
        self.audit_frames = E.plan_array(self.buf, p.audit_frames, p.n_audit, torch.int32)
        ga = geo16.with_frames(p.n_audit)
        self.Ka = E.frames_tensor(ga)
        if p.n_audit:
            E.emc_pack_frames_list(ga, counts_dev, self.audit_frames, self.Ka)
        self.ws = torch.empty(E.emc_proposed_workspace_bytes(geo16, p), dtype=torch.uint8, device="cuda")
        self.loglik = torch.empty(1, dtype=torch.float64, device="cuda")
        self.recall = torch.empty(1, dtype=torch.float64, device="cuda")

    def candidate_pairs(self) -> int:
        """(rotation, frame) pairs the candidate E-step evaluates: the rotations of every
        proposed cell of every candidate frame (synchronises)."""
        p = self.plan
        cells = E.plan_array(self.buf, p.cand_cells, p.n_cand * p.k_top, torch.int32).long()
        ptr = E.plan_array(self.buf, p.cell_ptr, p.n_cells + 1, torch.int64)
        return int((ptr[1:] - ptr[:-1])[cells[cells >= 0]].sum().item())

    def computed_pairs(self) -> int:
        """(rotation, frame) pairs the candidate log-likelihood and M-step compute: every
        rotation of a pack of cells over the union of its cells' frame lists (synchronises)."""
        p = self.plan
        groups = E.plan_array(self.buf, p.groups, 4 * p.n_groups, torch.int32).view(-1, 4).long()
        cf_ptr = E.plan_array(self.buf, p.cf_ptr, p.n_cells + 1, torch.int64)
        F = cf_ptr[1:] - cf_ptr[:-1]
        return int((groups[:, 2] * F[groups[:, 0]]).sum().item())

    def step(self, model_in, model_out, stage_events=None):
        E.emc_iterate_proposed(self.geo, self.plan, self.Ka, model_in, model_out, self.loglik, self.recall, self.ws,
                               stage_events)

    def accepted(self) -> bool:
        """The audit's verdict on the last step (synchronises).  Without audited
        frames there is no verdict (accepted); with them, a recall that is not a
        number (a broken iteration) rejects."""
        rec = self.recall.item()
        if self.plan.n_audit == 0:
            return True
        return math.isfinite(rec) and rec >= RECALL_MIN

    def view(self):
        """Workspace offsets of the last step's candidate G, P, b, L, S (see
        emc_proposed_workspace_view)."""
        return E.emc_proposed_workspace_view(self.geo, self.plan)


def proposal_lists(geo: E.Geometry, P, cells: CellIndex, n_cells: int, top_net, k_net: int, k_prev: int):
    """Each frame's proposal: the network's top-k_net cells (top_net [n_data][k_net], or
    None) followed by those of the k_prev cells holding most of the frame's mass in the
    full-search responsibilities P (emc_cell_targets, emc_cell_topk, emc_topk_union).
    Returns (lists [n_data * k], k)."""
    n = geo.n_data
    T = torch.empty(n * n_cells, dtype=torch.float32, device="cuda")
    E.emc_cell_targets(geo, P, cells.cell_ptr, cells.cell_rot, n_cells, T)
    top_prev = torch.empty(n * k_prev, dtype=torch.int32, device="cuda")
    E.emc_cell_topk(T, n, n_cells, k_prev, top_prev)
    if top_net is None:
        return top_prev, k_prev
    out = torch.empty(n * (k_net + k_prev), dtype=torch.int32, device="cuda")
    E.emc_topk_union(top_net, k_net, top_prev, k_prev, n, n_cells, out)
    return out, k_net + k_prev


def proposed_or_full(prop: ProposedIteration, full_step, model_in, model_out, stage_events=None) -> bool:
    """One iteration: the restricted one, judged by its audit; when the audit rejects
    it, the full search from the same model replaces its result
    (full_step(model_in, model_out) writes model_out).  Returns the verdict."""
    prop.step(model_in, model_out, stage_events)
    if prop.accepted():
        return True
    full_step(model_in, model_out)
    return False


class FullSearchChunks:
    """The full BF16 search over frame chunks of one problem (the fallback of a chunk
    whose audit rejects its proposal): one expansion per iteration, then for a chunk
    its frames packed, log-likelihoods, E-step and M/c-step added into num/den."""

    def __init__(self, geo16: E.Geometry, counts_dev, chunk: int):
        self.geo, self.counts, self.chunk = geo16, counts_dev, int(chunk)
        dev = "cuda"
        g = geo16.with_frames(self.chunk)
        ps, ds, nr = g.pix_stride, g.data_stride, g.n_rot
        self.frames = torch.arange(geo16.n_data, dtype=torch.int32, device=dev)
        self.K = E.frames_tensor(g)
        self.slices = E.slices_tensor(g)
        self.c = torch.empty(ps, dtype=torch.float64, device=dev)
        self.S = torch.empty(nr, dtype=torch.float64, device=dev)
        self.scale = torch.empty(nr, dtype=torch.float32, device=dev)
        self.G = torch.empty(nr * ds, dtype=torch.float32, device=dev)
        self.P = torch.empty(nr * ds, dtype=torch.bfloat16, device=dev)
        self.b = torch.empty(self.chunk, dtype=torch.float64, device=dev)
        self.stats = torch.empty(2 * self.chunk, dtype=torch.float64, device=dev)
        self.rho = torch.empty(nr, dtype=torch.float64, device=dev)
        self.Wp = torch.empty(nr * ps, dtype=torch.float32, device=dev)   # W' apart: the slices serve every chunk
        self.cws = torch.empty(E.emc_compress_workspace_bytes(g), dtype=torch.uint8, device=dev)
        self.expanded = None

    def bounds(self, ci: int):
        s = ci * self.chunk
        return s, min(self.geo.n_data, s + self.chunk)

    def expand(self, model):
        E.emc_expand(self.geo, model, self.c, self.slices, self.S, self.scale)
        self.expanded = model

    def add_chunk(self, ci: int, model, num, den, L, accumulate: bool):
        """Chunk ci's full search into num/den (zeroed first unless accumulate); its
        frames' log-evidence into L [chunk frames]; P of the chunk stays in self.P.
        The slices of the last expand() are reused while `model` is the same tensor:
        a caller that rewrites a model tensor in place calls expand() (or sets
        `expanded` to None) before the next chunk."""
        if self.expanded is not model:
            self.expand(model)
        s, e = self.bounds(ci)
        g = self.geo.with_frames(e - s)
        E.emc_pack_frames_list(g, self.counts, self.frames[s:e], self.K)
        E.emc_loglik(g, self.K, self.slices, self.scale, self.c, self.G, self.b)
        E.emc_responsibilities(g, self.G, self.S, self.b, E.EMC_RESP_FULL, self.stats, self.P, L, self.rho)
        E.emc_compress(g, self.P, self.K, self.rho, self.Wp, num, den, accumulate=accumulate, ws=self.cws)


def proposed_chunks(chunks, full: FullSearchChunks, model_in, model_out, loglik, L, num, den, make_plan,
                    recall_min: float = RECALL_MIN):
    """One iteration over frame chunks, the k-direction split of Section 3.3 applied to the
    restricted iteration: chunk ci's proposal (plan and audit from make_plan(ci), a
    ProposedIteration over that chunk's frames) adds its c-step sums into num/den when its
    audit accepts it; a rejected chunk adds the full search's sums instead.  One division
    (eq. 2.12) and the mean log-evidence (eq. 2.1) over every frame follow.
    Returns the audit recall of each chunk and whether it was accepted."""
    out = []
    full.expanded = None          # the first full-search chunk expands this iteration's model
    for ci in range(chunks):
        s, e = full.bounds(ci)
        prop = make_plan(ci)
        E.emc_proposed_accumulate(prop.geo, prop.plan, prop.Ka, model_in, num, den, ci > 0, recall_min, L[s:e],
                                  prop.recall, prop.ws)
        ok = prop.accepted()          # synchronises: the host decides the redo
        rec = prop.recall.item()
        if not ok:                    # the device gate added nothing for this chunk
            full.add_chunk(ci, model_in, num, den, L[s:e], accumulate=True)
        out.append((rec, ok))
        del prop
    E.emc_finalize(full.geo, num, den, model_in, model_out, L, full.geo.n_data, loglik)
    return out
