"""What the trained proposal network gains, on the 128^3 workload (16384 pixels,
25000 rotations, 100000 frames, ~2000 photons per frame) and its schedule: full
BF16 iterations 1-10, cell targets from iterations 8-10, two epochs of training,
then iteration 11 run from the same model with the full search (the reference)
and with proposals.

* recall: the trained network's top-64 of 2000 cells hold >= 0.98 of iteration
  11's posterior mass per frame, against about 64/2000 for the same network
  untrained;
* the learned form (network top-64 U the 64 cells of largest responsibility in
  iteration 10) is accepted by its audit and agrees with the full search within
  the learned-form tolerances: model relative L2 <= 1e-3; top-1 >= 99 % (the
  full search's most probable rotation lies in the frame's proposed cells, so
  the restricted posterior, the full one renormalised over the proposed
  rotations, has the same most probable rotation);
* the network's share: the same iteration with the previous posterior's cells
  alone has a larger model error than with the network's cells added.
"""
import numpy as np
import pytest

from emc_inputs import WORKLOADS, make_inputs, proposal_bins, shoemake_quaternions
from emc_inputs import rng as seeded

pytestmark = pytest.mark.gpu

N_CELLS, K_NET, K_PREV, TRAIN_AT = 2000, 64, 64, 10


def test_trained_proposal_gain(gpu_lib):
    import torch

    import bench
    from paper_1409_4256_amd import emc, learned

    wl = WORKLOADS[2]
    inp = make_inputs(wl, device="cuda", with_truth=False)
    run = bench.Run(inp, emc.EMC_PREC_BF16, inp.counts)
    g = run.geo
    coarse = torch.as_tensor(shoemake_quaternions(seeded(wl.cfg, "coarse"), N_CELLS), dtype=torch.float32,
                             device="cuda")
    cells = learned.CellIndex(g, coarse, N_CELLS)

    def targets_now():
        T = torch.empty(wl.n_data * N_CELLS, dtype=torch.float32, device="cuda")
        emc.emc_cell_targets(g, run.P, cells.cell_ptr, cells.cell_rot, N_CELLS, T)
        return T

    targets = []
    for it in range(TRAIN_AT):
        run.step()
        if it >= TRAIN_AT - 3:
            targets.append(targets_now())
    print(f"\n[gain] {TRAIN_AT} full iterations done", flush=True)
    bins = torch.as_tensor(proposal_bins(wl.det_n, inp.mask), device="cuda")
    init = learned.init_params(seeded(wl.cfg, "cnn"), N_CELLS)
    trained = learned.Network(N_CELLS, init.clone())
    untrained = learned.Network(N_CELLS, init.clone())
    x = trained.images(g, run.K, bins)
    tlog = trained.train(x, targets, wl.n_data, epochs=2, lr=1e-3, rng=seeded(wl.cfg, "cnn"))
    T_prev = targets[-1]
    del targets
    top_t = trained.topk(x, wl.n_data, K_NET)
    top_u = untrained.topk(x, wl.n_data, K_NET)
    del x
    top_prev = torch.empty(wl.n_data * K_PREV, dtype=torch.int32, device="cuda")
    emc.emc_cell_topk(T_prev, wl.n_data, N_CELLS, K_PREV, top_prev)
    union = torch.empty(wl.n_data * (K_NET + K_PREV), dtype=torch.int32, device="cuda")
    emc.emc_topk_union(top_t, K_NET, top_prev, K_PREV, wl.n_data, N_CELLS, union)
    print(f"[gain] trained in {tlog.seconds:.1f} s, loss {tlog.loss_first:.3f} -> {tlog.loss_last:.3f}", flush=True)

    m_in = run.model[run.cur].clone()
    run.step()                                               # iteration 11, full search
    T11 = targets_now().view(wl.n_data, N_CELLS)
    m_full = run.model[run.cur].double()
    best_full = run.P.view(wl.n_rot, -1)[:, :wl.n_data].float().argmax(0)
    r_t = torch.gather(T11, 1, top_t.view(-1, K_NET).long()).sum(1).mean().item()
    r_u = torch.gather(T11, 1, top_u.view(-1, K_NET).long()).sum(1).mean().item()
    del T11
    best_cell = cells.cell_of.long()[best_full]
    top1 = (union.view(-1, K_NET + K_PREV).long() == best_cell.unsqueeze(1)).any(1).float().mean().item()

    n_audit = int(round(0.02 * wl.n_data))
    audit = torch.as_tensor(np.sort(seeded(wl.cfg, "audit").choice(wl.n_data, n_audit, replace=False)),
                            dtype=torch.int32, device="cuda")

    def iterate(lists, k):
        prop = learned.ProposedIteration(g, inp.counts, coarse, N_CELLS, lists, k, audit)
        out = torch.empty_like(m_in)
        prop.step(m_in, out)                                 # iteration 11 with the proposal
        torch.cuda.synchronize()
        err = (torch.linalg.norm(out.double() - m_full) / torch.linalg.norm(m_full)).item()
        return err, prop.recall.item(), prop.accepted(), prop.candidate_pairs()

    err, rec, ok, pairs = iterate(union, K_NET + K_PREV)
    err_p, rec_p, _, pairs_p = iterate(top_prev, K_PREV)
    dense = wl.n_rot * wl.n_data
    print(f"[gain] recall of top-{K_NET}/{N_CELLS} cells: trained {r_t:.4f}, untrained {r_u:.4f}\n"
          f"[gain] learned form: model rel L2 vs full search {err:.2e}, top-1 {top1:.4f}, audit recall {rec:.5f}, "
          f"candidate pairs {pairs / dense:.4f} of dense\n"
          f"[gain] previous posterior's cells alone: model rel L2 {err_p:.2e}, audit recall {rec_p:.5f}, "
          f"pairs {pairs_p / dense:.4f} of dense", flush=True)
    assert r_t >= 0.98
    assert r_u <= 0.2
    assert ok
    assert err <= 1e-3
    assert top1 >= 0.99
    assert err < err_p
