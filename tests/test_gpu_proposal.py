"""Learned-proposal iteration on the GPU vs the FP64 oracle of the same restricted
E-step (implementation error) and vs the full-search oracle (approximation error).

Proposals here come from random logits: the restricted E-step, the plan and the
audit are checked independently of how good the network is."""
import numpy as np
import pytest

import oracle as O
from emc_inputs import shoemake_quaternions, tiny_problem
from oracle import cnn_oracle as C
from paper_1409_4256_amd import emc as E

pytestmark = pytest.mark.gpu


def _run(seed, N, npx, nrot, ndata, n_cells, k_top, n_audit, qr=None, photons=300.0):
    import torch

    from gpu_helpers import geometry, upload_counts

    t = tiny_problem(seed, grid_n=N, n_pix=npx, n_rot=nrot, n_data=ndata, photons=photons, q_radius=qr)
    q = np.asarray(t["q"], np.float32).astype(np.float64)
    quat = np.asarray(t["quat"], np.float32).astype(np.float64)
    rng = np.random.default_rng(100 + seed)
    coarse = np.asarray(shoemake_quaternions(rng, n_cells), np.float32)
    logits = rng.standard_normal((ndata, n_cells)).astype(np.float32)
    audit = np.sort(rng.choice(ndata, n_audit, replace=False)).astype(np.int32)
    geo = geometry(N, q, t["mask"], quat, t["log_w"], ndata, E.EMC_PREC_BF16)
    dev = "cuda"
    topk = torch.empty(ndata * k_top, dtype=torch.int32, device=dev)
    E.emc_cnn_topk(torch.as_tensor(logits, device=dev), ndata, n_cells, k_top, topk)
    counts = upload_counts(t["counts"])
    nz_cap = int((t["counts"] != 0).sum()) + 1
    buf = torch.empty(E.emc_proposal_bytes(geo, n_cells, k_top, n_audit, nz_cap), dtype=torch.uint8, device=dev)
    plan = E.emc_proposal_build(geo, torch.as_tensor(coarse, device=dev), n_cells, topk, k_top,
                                torch.as_tensor(audit, device=dev) if n_audit else None, counts, nz_cap, buf)
    cand_frames = E.plan_array(buf, plan.cand_frames, plan.n_cand, torch.int32)
    audit_frames = E.plan_array(buf, plan.audit_frames, plan.n_audit, torch.int32)
    gc, ga = geo.with_frames(plan.n_cand), geo.with_frames(plan.n_audit)
    Kc, Ka = E.frames_tensor(gc), E.frames_tensor(ga)
    if plan.n_cand:
        E.emc_pack_frames_list(gc, counts, cand_frames, Kc)
    if plan.n_audit:
        E.emc_pack_frames_list(ga, counts, audit_frames, Ka)
    cap = ndata * nrot  # every (rotation, frame) pair may be significant in these flat posteriors
    ws = torch.empty(E.emc_proposed_workspace_bytes(geo, plan, cap), dtype=torch.uint8, device=dev)
    m_in = torch.as_tensor(t["model"], dtype=torch.float32, device=dev)
    m_out = torch.empty_like(m_in)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    rec = torch.empty(1, dtype=torch.float64, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    E.emc_iterate_proposed(geo, plan, Kc, Ka, m_in, m_out, ll, rec, status, cap, ws)
    torch.cuda.synchronize()
    # oracle: the same candidate sets
    cell_of = C.assign_cells(coarse.astype(np.float64), coarse.astype(np.float64)) if False else \
        C.assign_cells(quat, coarse.astype(np.float64))
    top = C.topk_cells(logits.astype(np.float64), k_top)
    cand = np.zeros((nrot, ndata), bool)
    for k in range(ndata):
        cand[:, k] = np.isin(cell_of, top[k])
    cand_a = cand.copy()
    cand_a[:, audit] = True
    model = m_in.double().cpu().numpy()
    o = O.iterate_proposed(model, t["counts"], q, t["mask"], quat, t["log_w"], N, cand_a)
    full = O.iterate(model, t["counts"], q, t["mask"], quat, t["log_w"], N)
    recall_ref = O.proposal_recall(full["P"][:, audit], cand[:, audit]).mean() if n_audit else float("nan")
    return dict(plan=plan, buf=buf, cand_frames=cand_frames.cpu().numpy(), audit_frames=audit_frames.cpu().numpy(),
                model=m_out.double().cpu().numpy(), loglik=ll.item(), recall=rec.item(), status=status.item(),
                oracle=o, full=full, recall_ref=recall_ref, audit=audit, cell_of=cell_of, top=top,
                geo=geo)


@pytest.mark.parametrize("seed,N,npx,nrot,ndata,n_cells,k_top,n_audit",
                         [(0, 20, 300, 700, 600, 40, 8, 12), (1, 16, 200, 400, 300, 17, 3, 0),
                          (2, 24, 400, 1100, 520, 64, 20, 30)])
def test_proposed_iteration_matches_restricted_oracle(gpu_lib, seed, N, npx, nrot, ndata, n_cells, k_top, n_audit):
    from gpu_helpers import rel_l2

    r = _run(seed, N, npx, nrot, ndata, n_cells, k_top, n_audit)
    assert r["status"] == 0
    # plan: every frame exactly once, audited frames apart
    got = np.sort(np.concatenate([r["cand_frames"], r["audit_frames"]]))
    np.testing.assert_array_equal(got, np.arange(ndata))
    np.testing.assert_array_equal(np.sort(r["audit_frames"]), r["audit"])
    # implementation error vs the FP64 oracle of the same restricted E-step (BF16 form)
    err = rel_l2(r["model"], r["oracle"]["model"])
    print(f"\n[proposal seed{seed}] model rel L2 vs restricted oracle {err:.2e}, "
          f"vs full search {rel_l2(r['model'], r['full']['model']):.2e}")
    assert err <= 1e-3
    assert abs(r["loglik"] - r["oracle"]["loglik"]) <= 1e-3 * abs(r["oracle"]["loglik"])
    if n_audit:
        assert abs(r["recall"] - r["recall_ref"]) <= 1e-3, (r["recall"], r["recall_ref"])


def test_proposal_with_every_cell_is_full_search(gpu_lib):
    """k_top = n_cells makes every rotation a candidate: the result is the full search."""
    from gpu_helpers import rel_l2

    r = _run(4, 18, 250, 500, 400, 12, 12, 10)
    assert r["status"] == 0
    assert rel_l2(r["model"], r["full"]["model"]) <= 1e-3
    assert abs(r["recall"] - 1.0) <= 4e-3   # sum of BF16-rounded responsibilities
