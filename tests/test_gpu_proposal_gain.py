"""What the trained proposal network gains over the method without it.

Workload: the 128^3-share physics at a 64x64 detector and 64^3 grid (4000
rotations, 20000 frames, ~2000 photons), started from the true model so that
EMC's posteriors are concentrated from the first iteration; the schedule is the
specified one: full BF16 iterations 1-3 give the targets, the network is
trained on them, iteration 4 runs with the proposal (2 % audited).

* recall of the trained network's top-K cells on iteration 4's full posterior
  >= 0.98, against ~K / n_cells for the untrained network;
* the proposal-form iteration agrees with the full-search iteration from the
  same model within the learned-form tolerances (model relative L2 <= 1e-3,
  top-1 orientation agreement >= 99 %);
* the candidate work is reported as a fraction of the dense work, and the
  iteration times side by side.
"""
import numpy as np
import pytest

from emc_inputs import WORKLOADS, make_inputs, proposal_bins, scaled, shoemake_quaternions

pytestmark = pytest.mark.gpu

N_CELLS, K_TOP = 400, 16


def test_trained_proposal_gain(gpu_lib):
    import torch

    import bench
    from paper_1409_4256_amd import emc, learned

    wl = scaled(WORKLOADS[2], grid_n=64, det_n=64, n_rot=4000, n_data=20000, pool=2000, mask="random5")
    inp = make_inputs(wl, device="cuda", with_truth=True)
    inp.model_start = inp.model_true                       # concentrated posteriors from iteration 1
    run = bench.Run(inp, emc.EMC_PREC_BF16, inp.counts)
    g = run.geo
    rng = np.random.default_rng(1409)
    coarse = torch.as_tensor(shoemake_quaternions(rng, N_CELLS), dtype=torch.float32, device="cuda")
    cells = learned.CellIndex(g, coarse, N_CELLS)
    targets = []
    for it in range(3):
        run.step()
        T = torch.empty(wl.n_data * N_CELLS, dtype=torch.float32, device="cuda")
        emc.emc_cell_targets(g, run.P, cells.cell_ptr, cells.cell_rot, N_CELLS, T)
        targets.append(T)
    bins = torch.as_tensor(proposal_bins(wl.det_n, inp.mask), device="cuda")
    trained = learned.Network(N_CELLS, learned.init_params(np.random.default_rng(8), N_CELLS))
    x = trained.images(g, run.K, bins)
    log = trained.train(x, targets, wl.n_data, epochs=4, lr=1e-3, rng=np.random.default_rng(9))
    untrained = learned.Network(N_CELLS, learned.init_params(np.random.default_rng(8), N_CELLS))
    top_t = trained.topk(x, wl.n_data, K_TOP)
    top_u = untrained.topk(x, wl.n_data, K_TOP)
    # iteration 4: full search from the current model (reference) ...
    m_in = run.model[run.cur].clone()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    run.step()
    ev[1].record()
    T4 = torch.empty(wl.n_data * N_CELLS, dtype=torch.float32, device="cuda")
    emc.emc_cell_targets(g, run.P, cells.cell_ptr, cells.cell_rot, N_CELLS, T4)
    P_full = run.P.view(wl.n_rot, -1)[:, :wl.n_data].float()
    m_full = run.model[run.cur].double()

    def recall(top):
        return torch.gather(T4.view(wl.n_data, N_CELLS), 1, top.view(wl.n_data, K_TOP).long()).sum(1).mean().item()

    r_t, r_u = recall(top_t), recall(top_u)
    # ... and with the trained proposal
    n_audit = int(round(0.02 * wl.n_data))
    audit = torch.as_tensor(np.sort(rng.choice(wl.n_data, n_audit, replace=False)), dtype=torch.int32, device="cuda")
    prop = learned.ProposedIteration(g, inp.counts, coarse, N_CELLS, top_t, K_TOP, audit, 64 * wl.n_data)
    m_out = torch.empty_like(m_in)
    prop.step(m_in, m_out)          # warm-up
    ev[2].record()
    prop.step(m_in, m_out)
    ev[3].record()
    torch.cuda.synchronize()
    t_full, t_prop = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
    model_err = (torch.linalg.norm(m_out.double() - m_full) / torch.linalg.norm(m_full)).item()
    # top-1 orientation: the proposal form's best rotation per frame vs the full search's
    cand_frames = emc.plan_array(prop.buf, prop.plan.cand_frames, prop.plan.n_cand, torch.int64
                                 if False else torch.int32).long()
    best_full = P_full.argmax(0)
    # the proposal's best rotation of each candidate frame is the full search's best if it lies
    # in the frame's candidate cells and the restricted posterior is the conditional posterior
    cell_of = cells.cell_of.long()
    in_cand = (cell_of[best_full][cand_frames].unsqueeze(1) == top_t.view(wl.n_data, K_TOP)[cand_frames].long()).any(1)
    top1 = in_cand.float().mean().item()
    print(f"\n[gain] trained recall {r_t:.4f} vs untrained {r_u:.4f} (K/n_cells {K_TOP / N_CELLS:.3f}); "
          f"audit recall {prop.recall.item():.4f}; model rel L2 vs full search {model_err:.2e}; top-1 {top1:.4f}; "
          f"candidate pairs {prop.plan.n_g / (wl.n_rot * wl.n_data):.3f} of dense; "
          f"iteration {t_prop:.1f} ms proposal vs {t_full:.1f} ms full; training {log.seconds:.1f} s, "
          f"loss {log.loss_first:.2f} -> {log.loss_last:.2f}")
    assert prop.accepted()
    assert r_t >= 0.98
    assert r_u <= 0.3
    assert model_err <= 1e-3
    assert top1 >= 0.99
