"""Learned-proposal iteration on the GPU vs the FP64 oracle of the same restricted
E-step (implementation error) and vs the full-search oracle (approximation error).

Proposals here come from random logits (optionally merged with a second random
list and cut to ragged lengths): the restricted E-step, the plan and the audit
are checked independently of how good the network is."""
import numpy as np
import pytest

import oracle as O
from emc_inputs import shoemake_quaternions, tiny_problem
from oracle import cnn_oracle as C
from paper_1409_4256_amd import emc as E

pytestmark = pytest.mark.gpu


def _lists(rng, ndata, n_cells, k_top, k_extra, ragged):
    """Proposal lists [ndata][k_top + k_extra]: top-k_top of random logits, then the
    cells of a second random top-k_extra list not already present, -1 padding; with
    `ragged`, every row keeps only a random-length prefix of its valid entries."""
    logits = rng.standard_normal((ndata, n_cells))
    out = np.full((ndata, k_top + k_extra), -1, np.int32)
    for k in range(ndata):
        row = list(C.topk_cells(logits[k:k + 1], k_top)[0])
        if k_extra:
            other = C.topk_cells(rng.standard_normal((1, n_cells)), k_extra)[0]
            row += [c for c in other if c not in row]
        if ragged:
            row = row[:rng.integers(1, len(row) + 1)]
        out[k, :len(row)] = row
    return out


def _run(seed, N, npx, nrot, ndata, n_cells, k_top, n_audit, qr=None, photons=300.0, k_extra=0, ragged=False,
         brick=False):
    import torch

    from gpu_helpers import geometry, upload_counts

    t = tiny_problem(seed, grid_n=N, n_pix=npx, n_rot=nrot, n_data=ndata, photons=photons, q_radius=qr)
    q = np.asarray(t["q"], np.float32).astype(np.float64)
    quat = np.asarray(t["quat"], np.float32).astype(np.float64)
    rng = np.random.default_rng(100 + seed)
    coarse = np.asarray(shoemake_quaternions(rng, n_cells), np.float32)
    lists = _lists(rng, ndata, n_cells, k_top, k_extra, ragged)
    kk = lists.shape[1]
    audit = np.sort(rng.choice(ndata, n_audit, replace=False)).astype(np.int32)
    geo = geometry(N, q, t["mask"], quat, t["log_w"], ndata, E.EMC_PREC_BF16)
    if brick:
        geo.use_brick_scatter(chunk=64)
    dev = "cuda"
    topk = torch.as_tensor(lists.reshape(-1), device=dev)
    counts = upload_counts(t["counts"])
    nz_cap = int((t["counts"] != 0).sum()) + 1
    print(f"[proposal] seed {seed} N {N} npx {npx} nrot {nrot} ndata {ndata} cells {n_cells} list {kk} "
          f"audit {n_audit}", flush=True)
    buf = torch.empty(E.emc_proposal_bytes(geo, n_cells, kk, n_audit, nz_cap), dtype=torch.uint8, device=dev)
    plan = E.emc_proposal_build(geo, torch.as_tensor(coarse, device=dev), n_cells, topk, kk,
                                torch.as_tensor(audit, device=dev) if n_audit else None, counts, nz_cap, buf)
    cand_frames = E.plan_array(buf, plan.cand_frames, plan.n_cand, torch.int32)
    audit_frames = E.plan_array(buf, plan.audit_frames, plan.n_audit, torch.int32)
    ga = geo.with_frames(plan.n_audit)
    Ka = E.frames_tensor(ga)
    if plan.n_audit:
        E.emc_pack_frames_list(ga, counts, audit_frames, Ka)
    ws = torch.empty(E.emc_proposed_workspace_bytes(geo, plan), dtype=torch.uint8, device=dev)
    m_in = torch.as_tensor(t["model"], dtype=torch.float32, device=dev)
    m_out = torch.empty_like(m_in)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    rec = torch.empty(1, dtype=torch.float64, device=dev)
    E.emc_iterate_proposed(geo, plan, Ka, m_in, m_out, ll, rec, ws)
    torch.cuda.synchronize()
    # candidate pairs' log-likelihood sums and responsibilities, read from the workspace
    from gpu_helpers import candidate_pairs, proposed_pairs_values

    view = E.emc_proposed_workspace_view(geo, plan)
    pairs = candidate_pairs(buf, plan, nrot)
    Gv, Pv = proposed_pairs_values(ws, view, pairs)
    f64 = lambda off, n: ws[off:off + 8 * n].view(torch.float64).cpu().numpy()
    order = np.concatenate([cand_frames.cpu().numpy(), audit_frames.cpu().numpy()]).astype(np.int64)
    b_frame = np.empty(ndata)
    b_frame[order] = f64(view.b, ndata)
    L_frame = np.empty(ndata)
    L_frame[order] = f64(view.L, ndata)
    S_dev = f64(view.S, nrot)
    na, dsa = plan.n_audit, E.emc_data_stride(plan.n_audit)
    Pa = ws[view.Pa:view.Pa + 2 * nrot * dsa].view(torch.bfloat16).view(nrot, dsa)[:, :na].double().cpu().numpy() \
        if na else np.zeros((nrot, 0))
    # oracle: the same candidate sets
    cell_of = C.assign_cells(quat, coarse.astype(np.float64))
    cand = np.zeros((nrot, ndata), bool)
    for k in range(ndata):
        cand[:, k] = np.isin(cell_of, lists[k][lists[k] >= 0])
    cand_a = cand.copy()
    cand_a[:, audit] = True
    model = m_in.double().cpu().numpy()
    o = O.iterate_proposed(model, t["counts"], q, t["mask"], quat, t["log_w"], N, cand_a)
    full = O.iterate(model, t["counts"], q, t["mask"], quat, t["log_w"], N)
    recall_ref = O.proposal_recall(full["P"][:, audit], cand[:, audit]).mean() if n_audit else float("nan")
    j, k = pairs[0], pairs[1]
    return dict(plan=plan, buf=buf, cand_frames=cand_frames.cpu().numpy(), audit_frames=audit_frames.cpu().numpy(),
                model=m_out.double().cpu().numpy(), loglik=ll.item(), recall=rec.item(),
                oracle=o, full=full, recall_ref=recall_ref, audit=audit, cell_of=cell_of, lists=lists, geo=geo,
                cand=cand, pair_j=j, pair_k=k, pair_Q=Gv + b_frame[k] - S_dev[j], pair_P=Pv, L_frame=L_frame, Pa=Pa)


def _check_restricted(r, ndata, tag):
    from gpu_helpers import rel_l2

    # plan: every frame exactly once, audited frames apart
    got = np.sort(np.concatenate([r["cand_frames"], r["audit_frames"]]))
    np.testing.assert_array_equal(got, np.arange(ndata))
    np.testing.assert_array_equal(np.sort(r["audit_frames"]), r["audit"])
    # implementation error vs the FP64 oracle of the same restricted E-step (BF16 form)
    err = rel_l2(r["model"], r["oracle"]["model"])
    print(f"\n[proposal {tag}] model rel L2 vs restricted oracle {err:.2e}, "
          f"vs full search {rel_l2(r['model'], r['full']['model']):.2e}, loglik {r['loglik']:.6f} "
          f"(oracle {r['oracle']['loglik']:.6f})")
    assert err <= 1e-3
    assert abs(r["loglik"] - r["oracle"]["loglik"]) <= 1e-3 * abs(r["oracle"]["loglik"])
    if len(r["audit"]):
        assert abs(r["recall"] - r["recall_ref"]) <= 1e-3, (r["recall"], r["recall_ref"])
    _check_pairs(r, tag)


def _check_pairs(r, tag):
    """Element by element: every candidate pair's log-likelihood Q_jk = G + b_k - S_j
    (eq. 2.3) and responsibility (eq. 2.4 restricted to the candidates) against the
    oracle's, the pair set against the oracle's candidate matrix, and the audited
    frames' full-search responsibilities and every frame's log-evidence."""
    o = r["oracle"]
    j, k = r["pair_j"], r["pair_k"]
    cf = r["cand_frames"]
    # the candidate pairs are exactly the oracle's candidate set of the candidate frames
    assert j.size == int(r["cand"][:, cf].sum())
    assert np.all(r["cand"][j, k])
    assert np.unique(j * 10 ** 7 + k).size == j.size
    Qref = o["Q"][j, k]
    qscale = np.max(np.abs(o["Q"]), axis=0)[k]
    qerr = float(np.max(np.abs(r["pair_Q"] - Qref) / qscale)) if j.size else 0.0
    Pref = o["P"][j, k]
    perr = np.abs(r["pair_P"] - Pref)
    pexcess = float(np.max(perr - 2.0 ** -8 * Pref)) if j.size else 0.0
    Lerr = float(np.max(np.abs(r["L_frame"] - o["L"]) / np.abs(o["L"])))
    print(f"[proposal {tag}] {j.size} candidate pairs: Q rel err {qerr:.2e}, P max-abs err "
          f"{float(perr.max()) if j.size else 0.0:.2e} (beyond BF16 rounding {pexcess:.2e}), L rel err {Lerr:.2e}")
    assert qerr <= 2e-4
    # P is stored in BF16: its rounding (2^-9 relative) plus 1e-3
    assert pexcess <= 1e-3
    assert Lerr <= 2e-4
    a = r["audit_frames"]
    if a.size:
        pa = np.abs(r["Pa"] - o["P"][:, a])
        assert float(np.max(pa - 2.0 ** -8 * o["P"][:, a])) <= 1e-3


@pytest.mark.parametrize("seed,N,npx,nrot,ndata,n_cells,k_top,n_audit",
                         [(0, 20, 300, 700, 600, 40, 8, 12), (1, 16, 200, 400, 300, 17, 3, 0),
                          (2, 24, 400, 1100, 520, 64, 20, 30)])
def test_proposed_iteration_matches_restricted_oracle(gpu_lib, seed, N, npx, nrot, ndata, n_cells, k_top, n_audit):
    r = _run(seed, N, npx, nrot, ndata, n_cells, k_top, n_audit)
    _check_restricted(r, ndata, f"seed{seed}")


def test_union_lists_ragged_and_multi_group_cells(gpu_lib):
    """Lists merged from two proposals with -1 padding and ragged lengths; 10 cells
    over 1000 rotations put ~100 rotations (four groups of up to 32) in each cell."""
    r = _run(5, 20, 300, 1000, 500, 10, 3, 20, k_extra=3, ragged=True)
    _check_restricted(r, 500, "union/ragged/multi-group")
    assert r["plan"].n_groups > r["plan"].n_cells


def test_brick_major_compress(gpu_lib):
    """The proposal iteration with the brick-major c-step."""
    r = _run(0, 20, 300, 700, 600, 40, 8, 12, brick=True)
    _check_restricted(r, 600, "brick-major c-step")


def test_sparse_bands_only(gpu_lib):
    """~40 photons per frame: no band is dense, the M-step is the sparse path alone."""
    r = _run(8, 20, 300, 700, 500, 40, 8, 12, photons=40.0)
    assert r["plan"].n_dense == 0
    _check_restricted(r, 500, "sparse bands only")


def test_dense_bands(gpu_lib):
    """~3000 photons over 300 pixels: most pixels of a 128-pixel band are non-zero in
    every frame (more entries per band than a wave has lanes)."""
    r = _run(6, 20, 300, 600, 400, 24, 6, 16, photons=3000.0)
    assert 0 < r["plan"].n_dense < r["plan"].n_bands   # the padding band past n_pix stays sparse (empty)
    _check_restricted(r, 400, "dense bands")


@pytest.mark.parametrize("seed,nrot,n_cells,k_top", [(11, 700, 40, 8), (12, 1000, 10, 3), (13, 300, 120, 12)])
def test_plan_packs_and_lists_are_consistent(gpu_lib, seed, nrot, n_cells, k_top):
    """The plan's packs of cells, against numpy: every cell in exactly one pack, a
    pack holding at most 16 rotations unless it is a single cell; the pack-order
    rotation list a permutation holding each cell's rotations at cell_first, with
    the cell's index inside its pack; the groups tiling each pack's rotations in
    runs of at most 32; each pack's list holding exactly the candidate frames that
    propose one of its cells, each once, with the bits of those cells; and every
    list entry's column pointing at its frame in its cell's pack list.  The three
    cases have about 17, 100 (groups of 32 in one-cell packs) and 2.5 rotations per
    cell (many cells without a rotation)."""
    import torch

    from gpu_helpers import geometry, upload_counts

    t = tiny_problem(seed, grid_n=16, n_pix=200, n_rot=nrot, n_data=300, photons=200.0)
    q = np.asarray(t["q"], np.float32).astype(np.float64)
    quat = np.asarray(t["quat"], np.float32).astype(np.float64)
    rng = np.random.default_rng(200 + seed)
    coarse = np.asarray(shoemake_quaternions(rng, n_cells), np.float32)
    lists = _lists(rng, 300, n_cells, k_top, 2, True)
    kk = lists.shape[1]
    audit = np.sort(rng.choice(300, 9, replace=False)).astype(np.int32)
    geo = geometry(16, q, t["mask"], quat, t["log_w"], 300, E.EMC_PREC_BF16)
    counts = upload_counts(t["counts"])
    nz_cap = int((t["counts"] != 0).sum()) + 1
    buf = torch.empty(E.emc_proposal_bytes(geo, n_cells, kk, 9, nz_cap), dtype=torch.uint8, device="cuda")
    plan = E.emc_proposal_build(geo, torch.as_tensor(coarse, device="cuda"), n_cells,
                                torch.as_tensor(lists.reshape(-1), device="cuda"), kk,
                                torch.as_tensor(audit, device="cuda"), counts, nz_cap, buf)
    pa = lambda addr, n, dt=torch.int32: E.plan_array(buf, addr, n, dt).cpu().numpy().astype(np.int64)
    n_packs, nc = plan.n_packs, plan.n_cand
    cell_of = pa(plan.cell_of, nrot)
    # the GPU assigns cells in FP32: any cell within FP32 rounding of the best is a tie
    qn = quat / np.linalg.norm(quat, axis=1, keepdims=True)
    cn = coarse.astype(np.float64) / np.linalg.norm(coarse.astype(np.float64), axis=1, keepdims=True)
    dots = np.abs(qn @ cn.T)
    assert np.all(dots.max(axis=1) - dots[np.arange(nrot), cell_of] <= 1e-6)
    R = np.bincount(cell_of, minlength=n_cells)
    pack_of = pa(plan.pack_of, n_cells)
    cell_first = pa(plan.cell_first, n_cells)
    pack_rot = pa(plan.pack_rot, nrot)
    rot_local = pa(plan.rot_local, nrot)
    assert 1 <= n_packs <= n_cells and pack_of.min() == 0 and pack_of.max() == n_packs - 1
    assert np.all(np.bincount(pack_of, minlength=n_packs) > 0)
    np.testing.assert_array_equal(np.sort(pack_rot), np.arange(nrot))
    members = [np.flatnonzero(pack_of == p) for p in range(n_packs)]
    pack_start = np.zeros(n_packs, np.int64)
    local = np.full(n_cells, -1, np.int64)  # index inside the pack (known for cells with rotations)
    for p, cs in enumerate(members):
        assert cs.size == 1 or R[cs].sum() <= 16, (p, cs, R[cs])
        full = cs[R[cs] > 0]
        if full.size == 0:
            continue
        order = full[np.argsort(cell_first[full])]       # the pack's cells in their rotation order
        pack_start[p] = pos = cell_first[order[0]]
        for c in order:
            assert cell_first[c] == pos
            seg = pack_rot[pos:pos + R[c]]
            np.testing.assert_array_equal(np.sort(seg), np.flatnonzero(cell_of == c))
            li = rot_local[pos:pos + R[c]]
            assert np.all(li == li[0]) and 0 <= li[0] < cs.size
            local[c] = li[0]
            pos += R[c]
        assert np.unique(local[full]).size == full.size
    # groups: each pack's rotations in runs of at most 32, in order
    groups = pa(plan.groups, 4 * plan.n_groups).reshape(-1, 4)
    cg_ptr = pa(plan.cg_ptr, n_cells + 1, torch.int64)
    for p in range(n_packs):
        gs = groups[cg_ptr[p]:cg_ptr[p + 1]]
        total = R[members[p]].sum()
        assert np.all(gs[:, 0] == p) and np.all(gs[:, 2] <= 32) and gs[:, 2].sum() == total
        if total:
            np.testing.assert_array_equal(gs[:, 1], pack_start[p] + np.concatenate([[0], np.cumsum(gs[:-1, 2])]))
    # lists: exactly the frames proposing a cell of the pack, once, with that cell's bit
    cand_frames = pa(plan.cand_frames, nc)
    cells = pa(plan.cand_cells, nc * kk).reshape(nc, kk)
    np.testing.assert_array_equal(cells, lists[cand_frames])
    cf_ptr = pa(plan.cf_ptr, n_cells + 1, torch.int64)
    cf_frame = pa(plan.cf_frame, int(cf_ptr[n_packs]))
    cf_mask = pa(plan.cf_mask, int(cf_ptr[n_packs])) & 0xffffffff
    pair_col = pa(plan.pair_col, nc * kk).reshape(nc, kk)
    for p, cs in enumerate(members):
        fr = cf_frame[cf_ptr[p]:cf_ptr[p + 1]]
        want = np.flatnonzero(np.isin(cells, cs).any(axis=1))
        np.testing.assert_array_equal(np.sort(fr), want)
        m = cf_mask[cf_ptr[p]:cf_ptr[p + 1]]
        # one bit per proposed cell of the pack; a cell with rotations at its own index
        npro = np.isin(cells[fr], cs).sum(axis=1)
        np.testing.assert_array_equal(np.array([bin(int(x)).count("1") for x in m]), npro)
        for c in cs[R[cs] > 0]:
            np.testing.assert_array_equal((m >> local[c]) & 1, (cells[fr] == c).any(axis=1).astype(np.int64))
    f_idx, t_idx = np.nonzero(cells >= 0)
    p_of = pack_of[cells[f_idx, t_idx]]
    np.testing.assert_array_equal(cf_frame[cf_ptr[p_of] + pair_col[f_idx, t_idx]], f_idx)
    print(f"\n[proposal plan] {n_cells} cells in {n_packs} packs, {plan.n_groups} groups, "
          f"{int(cf_ptr[n_packs])} list entries for {int((cells >= 0).sum())} proposed (frame, cell) pairs")


def test_proposal_with_every_cell_is_full_search(gpu_lib):
    """k_top = n_cells makes every rotation a candidate: the result is the full search."""
    from gpu_helpers import rel_l2

    r = _run(4, 18, 250, 500, 400, 12, 12, 10)
    assert rel_l2(r["model"], r["full"]["model"]) <= 1e-3
    assert abs(r["recall"] - 1.0) <= 4e-3   # sum of BF16-rounded responsibilities


def test_counts_beyond_bf16_are_refused(gpu_lib):
    import torch

    from gpu_helpers import geometry, upload_counts

    t = tiny_problem(7, grid_n=16, n_pix=200, n_rot=300, n_data=50, photons=200.0)
    counts = t["counts"].copy()
    counts[3, np.flatnonzero(t["mask"])[0]] = 300
    geo = geometry(16, np.asarray(t["q"], np.float64), t["mask"], np.asarray(t["quat"], np.float64), t["log_w"], 50,
                   E.EMC_PREC_BF16)
    rng = np.random.default_rng(7)
    coarse = torch.as_tensor(np.asarray(shoemake_quaternions(rng, 8), np.float32), device="cuda")
    topk = torch.as_tensor(_lists(rng, 50, 8, 2, 0, False).reshape(-1), device="cuda")
    nz_cap = int((counts != 0).sum()) + 1
    buf = torch.empty(E.emc_proposal_bytes(geo, 8, 2, 0, nz_cap), dtype=torch.uint8, device="cuda")
    with pytest.raises(E.EmcError) as e:
        E.emc_proposal_build(geo, coarse, 8, topk, 2, None, upload_counts(counts), nz_cap, buf)
    assert e.value.status == E.EMC_ERR_RANGE


def test_cell_topk_and_union_match_numpy(gpu_lib):
    import torch

    rng = np.random.default_rng(11)
    rows, n_cells, k = 300, 150, 20
    T = rng.random((rows, n_cells)).astype(np.float32)
    T[T < 0.8] = 0.0                       # ~30 positive cells per row, some rows fewer than k
    T[5] = 0.0                             # a row with none
    T[7, :40] = 0.5                        # ties: lower index first
    out = torch.empty(rows * k, dtype=torch.int32, device="cuda")
    E.emc_cell_topk(torch.as_tensor(T, device="cuda"), rows, n_cells, k, out)
    got = out.view(rows, k).cpu().numpy()
    for r in range(rows):
        pos = np.flatnonzero(T[r] > 0)
        ref = pos[np.argsort(-T[r, pos], kind="stable")][:k]
        np.testing.assert_array_equal(got[r, :len(ref)], ref)
        assert (got[r, len(ref):] == -1).all()
    a = rng.integers(-1, n_cells, size=(rows, 12)).astype(np.int32)
    b = rng.integers(-1, n_cells, size=(rows, 70)).astype(np.int32)   # more than one wave of entries
    uo = torch.empty(rows * 82, dtype=torch.int32, device="cuda")
    E.emc_topk_union(torch.as_tensor(a, device="cuda"), 12, torch.as_tensor(b, device="cuda"), 70, rows, n_cells, uo)
    got = uo.view(rows, 82).cpu().numpy()
    for r in range(rows):
        ref = []
        for c in list(a[r]) + list(b[r]):
            if 0 <= c < n_cells and c not in ref:
                ref.append(int(c))
        np.testing.assert_array_equal(got[r, :len(ref)], ref)
        assert (got[r, len(ref):] == -1).all()


def test_audit_rejects_poor_proposal_and_full_search_replaces_it(gpu_lib):
    """Random two-cell proposals out of 40 hold far less than 0.98 of the audited
    frames' posterior mass: the audit rejects the restricted iteration, the full
    search from the same model replaces its result (equal to the FP64 oracle's full
    iteration within the BF16 tolerance), and the plan rebuilt from that full
    posterior proposes the cells of largest posterior mass and passes its audit."""
    import torch

    from gpu_helpers import geometry, rel_l2, upload_counts
    from paper_1409_4256_amd import learned

    N, npx, nrot, ndata, n_cells, n_audit = 20, 300, 700, 400, 40, 20
    t = tiny_problem(9, grid_n=N, n_pix=npx, n_rot=nrot, n_data=ndata, photons=3000.0)
    q = np.asarray(t["q"], np.float32).astype(np.float64)
    quat = np.asarray(t["quat"], np.float32).astype(np.float64)
    rng = np.random.default_rng(109)
    coarse = np.asarray(shoemake_quaternions(rng, n_cells), np.float32)
    lists = _lists(rng, ndata, n_cells, 2, 0, False)
    audit = np.sort(rng.choice(ndata, n_audit, replace=False)).astype(np.int32)
    geo = geometry(N, q, t["mask"], quat, t["log_w"], ndata, E.EMC_PREC_BF16)
    dev = "cuda"
    counts = upload_counts(t["counts"])
    coarse_d = torch.as_tensor(coarse, device=dev)
    audit_d = torch.as_tensor(audit, device=dev)
    print(f"[fallback] N {N} npx {npx} nrot {nrot} ndata {ndata} cells {n_cells}", flush=True)
    prop = learned.ProposedIteration(geo, counts, coarse_d, n_cells, torch.as_tensor(lists.reshape(-1), device=dev),
                                     2, audit_d)
    K = E.frames_tensor(geo)
    E.emc_pack_frames(geo, counts, K)
    ws_full = torch.empty(E.emc_workspace_bytes(geo), dtype=torch.uint8, device=dev)
    P_full = torch.empty(nrot * geo.data_stride, dtype=torch.bfloat16, device=dev)
    ll_full = torch.empty(1, dtype=torch.float64, device=dev)
    calls = []

    def full(a, b):
        calls.append(1)
        E.emc_iterate(geo, a, K, b, ll_full, P_out=P_full, ws=ws_full)

    m_in = torch.as_tensor(t["model"], dtype=torch.float32, device=dev)
    m_out = torch.empty_like(m_in)
    ok = learned.proposed_or_full(prop, full, m_in, m_out)
    torch.cuda.synchronize()
    model = m_in.double().cpu().numpy()
    o = O.iterate(model, t["counts"], q, t["mask"], quat, t["log_w"], N)
    cell_of = C.assign_cells(quat, coarse.astype(np.float64))
    cand = np.zeros((nrot, ndata), bool)
    for k in range(ndata):
        cand[:, k] = np.isin(cell_of, lists[k][lists[k] >= 0])
    rec_ref = O.proposal_recall(o["P"][:, audit], cand[:, audit]).mean()
    err = rel_l2(m_out.double().cpu().numpy(), o["model"])
    print(f"[fallback] audit recall {prop.recall.item():.4f} (oracle {rec_ref:.4f}), verdict {ok}; "
          f"model after the full search: rel L2 vs oracle {err:.2e}", flush=True)
    assert rec_ref < 0.98 and abs(prop.recall.item() - rec_ref) <= 1e-3
    assert not ok and len(calls) == 1
    assert err <= 1e-3
    # the plan rebuilt from the full posterior: the 8 cells of largest mass per frame
    cells = learned.CellIndex(geo, coarse_d, n_cells)
    new_lists, kk = learned.proposal_lists(geo, P_full, cells, n_cells, None, 0, 8)
    nl = new_lists.view(ndata, kk).cpu().numpy()
    T_ref = np.stack([o["P"][cell_of == c].sum(0) for c in range(n_cells)], axis=1)    # [frame][cell]
    best = np.sort(T_ref, axis=1)[:, ::-1][:, :8].sum(1)
    got = np.array([T_ref[f, nl[f][nl[f] >= 0]].sum() for f in range(ndata)])
    print(f"[fallback] rebuilt lists hold {got.mean():.5f} of the oracle posterior (best 8 cells: "
          f"{best.mean():.5f})", flush=True)
    assert np.all(got >= best - 2e-3)
    prop2 = learned.ProposedIteration(geo, counts, coarse_d, n_cells, new_lists, kk, audit_d)
    calls.clear()
    ok2 = learned.proposed_or_full(prop2, full, m_in, m_out)
    cand2 = np.zeros((nrot, ndata), bool)
    for k in range(ndata):
        cand2[:, k] = np.isin(cell_of, nl[k][nl[k] >= 0])
    rec2 = O.proposal_recall(o["P"][:, audit], cand2[:, audit]).mean()
    print(f"[fallback] rebuilt plan: audit recall {prop2.recall.item():.5f} (oracle {rec2:.5f}), verdict {ok2}",
          flush=True)
    assert abs(prop2.recall.item() - rec2) <= 1e-3
    assert rec2 >= 0.98 and ok2 and not calls



def test_streamed_chunks_with_audit_gate_match_oracle(gpu_lib):
    """Frame chunks of one restricted iteration (the k-direction split of Section 3.3),
    each with its own plan and audit, summed into one numerator and denominator before
    the division: chunks 0 and 2 propose each frame's 8 cells of largest oracle
    posterior mass and pass their audits; chunk 1 proposes 2 random cells, its audit
    rejects it, the device gate adds nothing for it and its full search is added
    instead.  The oracle: the restricted iteration's sums of the accepted chunks plus
    the full iteration's sums of the rejected one, divided once (eq. 2.4, 2.11-2.12)."""
    import torch

    from gpu_helpers import geometry, rel_l2, upload_counts
    from paper_1409_4256_amd import learned

    N, npx, nrot, n_cells, k_top = 20, 300, 700, 40, 8
    bounds = [(0, 250), (250, 500), (500, 600)]        # ragged last chunk
    ndata = bounds[-1][1]
    t = tiny_problem(12, grid_n=N, n_pix=npx, n_rot=nrot, n_data=ndata, photons=3000.0)
    q = np.asarray(t["q"], np.float32).astype(np.float64)
    quat = np.asarray(t["quat"], np.float32).astype(np.float64)
    rng = np.random.default_rng(112)
    coarse = np.asarray(shoemake_quaternions(rng, n_cells), np.float32)
    model = np.asarray(t["model"], np.float32).astype(np.float64)
    full = O.iterate(model, t["counts"], q, t["mask"], quat, t["log_w"], N)
    cell_of = C.assign_cells(quat, coarse.astype(np.float64))
    T = np.stack([full["P"][cell_of == c].sum(0) for c in range(n_cells)], axis=1)      # [frame][cell]
    good = np.argsort(-T, axis=1, kind="stable")[:, :k_top].astype(np.int32)
    lists = good.copy()
    lists[250:500] = -1
    lists[250:500, :2] = _lists(rng, 250, n_cells, 2, 0, False)
    audits = [np.sort(rng.choice(e - s, 10, replace=False)).astype(np.int32) for s, e in bounds]
    dev = "cuda"
    geo = geometry(N, q, t["mask"], quat, t["log_w"], ndata, E.EMC_PREC_BF16)
    counts = upload_counts(t["counts"])
    coarse_d = torch.as_tensor(coarse, device=dev)
    print(f"[streamed proposal] N {N} npx {npx} nrot {nrot} chunks {bounds}", flush=True)

    class Chunks(learned.FullSearchChunks):
        def bounds(self, ci):
            return bounds[ci]

    fc = Chunks(geo, counts, 250)

    def make_plan(ci):
        s, e = bounds[ci]
        return learned.ProposedIteration(geo.with_frames(e - s), counts[s:e], coarse_d, n_cells,
                                         torch.as_tensor(lists[s:e].reshape(-1), device=dev), k_top,
                                         torch.as_tensor(audits[ci], device=dev))

    M = N ** 3
    num = torch.full((M,), float("nan"), dtype=torch.float64, device=dev)   # the first chunk zeroes them
    den = torch.full((M,), float("nan"), dtype=torch.float64, device=dev)
    L = torch.empty(ndata, dtype=torch.float64, device=dev)
    m_in = torch.as_tensor(t["model"], dtype=torch.float32, device=dev)
    m_out = torch.empty_like(m_in)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    verdicts = learned.proposed_chunks(len(bounds), fc, m_in, m_out, ll, L, num, den, make_plan)
    torch.cuda.synchronize()
    # oracle, chunk by chunk
    num_o, den_o, L_o, rec_o = np.zeros(M), np.zeros(M), [], []
    for ci, (s, e) in enumerate(bounds):
        cand = np.zeros((nrot, e - s), bool)
        for k in range(e - s):
            row = lists[s + k]
            cand[:, k] = np.isin(cell_of, row[row >= 0])
        rec_o.append(float(O.proposal_recall(full["P"][:, s:e][:, audits[ci]], cand[:, audits[ci]]).mean()))
        if rec_o[-1] >= learned.RECALL_MIN:
            cand[:, audits[ci]] = True
            o = O.iterate_proposed(model, t["counts"][s:e], q, t["mask"], quat, t["log_w"], N, cand)
        else:
            o = O.iterate(model, t["counts"][s:e], q, t["mask"], quat, t["log_w"], N)
        num_o += o["num"]
        den_o += o["den"]
        L_o.append(o["L"])
    m_ref = O.divide(num_o, den_o, model)
    ll_ref = float(np.concatenate(L_o).mean())
    err = rel_l2(m_out.double().cpu().numpy(), m_ref)
    print(f"[streamed proposal] verdicts {verdicts}, oracle recalls {[round(r, 5) for r in rec_o]}; "
          f"model rel L2 vs oracle {err:.2e}, loglik {ll.item():.6f} (oracle {ll_ref:.6f})", flush=True)
    assert [ok for _, ok in verdicts] == [True, False, True]
    assert rec_o[0] >= 0.99 and rec_o[2] >= 0.99 and rec_o[1] < 0.9     # verdicts far from the bar
    for (rec, _), r in zip(verdicts, rec_o):
        assert abs(rec - r) <= 1e-3
    assert err <= 1e-3
    assert abs(ll.item() - ll_ref) <= 1e-3 * abs(ll_ref)
    assert torch.isfinite(num).all() and torch.isfinite(den).all()
