"""Helpers for the GPU parity tests: run the C-ABI entry points on device tensors
and bring every intermediate back as float64 numpy arrays in the oracle's index
order (rotation j, frame k, pixel i)."""
from __future__ import annotations

import numpy as np
import torch

from paper_1409_4256_amd import emc


def geometry(grid_n, q, mask, quat, log_w, n_data, precision=emc.EMC_PREC_FP32):
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dt)
    return emc.Geometry(grid_n, t(q, torch.float64), t(mask, torch.uint8), t(quat, torch.float64),
                        t(log_w, torch.float64), n_data, precision)


def upload_counts(counts):
    if isinstance(counts, torch.Tensor):
        return counts.to("cuda").contiguous()
    return torch.from_numpy(np.ascontiguousarray(counts.astype(np.uint16))).to("cuda")


def pack(geo, counts_dev):
    K = emc.frames_tensor(geo)
    emc.emc_pack_frames(geo, counts_dev, K)
    return K


def _slices_f64(geo, slices, scale):
    """Centred log slices A_ji as float64 [n_rot][ps] (hi + lo rescaled in BF16 form)."""
    nr, ps = geo.n_rot, geo.pix_stride
    if not geo.bf16:
        return slices[:nr * ps].view(nr, ps).double()
    hl = slices.view(torch.bfloat16)
    hi = hl[:nr * ps].view(nr, ps).double()
    lo = hl[nr * ps:2 * nr * ps].view(nr, ps).double()
    return (hi + lo) * scale.double()[:, None]


def run_steps(geo, model, K, frame_chunks=None, grid_copies=True):
    """expand -> loglik -> responsibilities -> compress -> finalize.

    `frame_chunks` is a list of (geometry, K_packed, offset) per chunk of frames
    (each packed on its own); None runs the whole frame set at once."""
    dev = "cuda"
    N3 = geo.grid_n ** 3
    ps = geo.pix_stride
    m = torch.as_tensor(np.asarray(model, dtype=np.float32)).to(dev)
    c = torch.empty(ps, dtype=torch.float64, device=dev)
    slices = emc.slices_tensor(geo)
    S = torch.empty(geo.n_rot, dtype=torch.float64, device=dev)
    scale = torch.empty(geo.n_rot, dtype=torch.float32, device=dev)
    emc.emc_expand(geo, m, c, slices, S, scale)
    out = dict(c=c, A=_slices_f64(geo, slices, scale), S=S, scale=scale)
    chunks = frame_chunks or [(geo, K, 0)]
    num = torch.empty(N3, dtype=torch.float64, device=dev)
    den = torch.empty(N3, dtype=torch.float64, device=dev)
    Wp = torch.empty(geo.n_rot * ps, dtype=torch.float32, device=dev)
    cws = torch.empty(emc.emc_compress_workspace_bytes(geo), dtype=torch.uint8, device=dev) if grid_copies else None
    n = geo.n_data
    Gs, Ps, bs, Ls, sts = [], [], [], [], []
    rho_tot = torch.zeros(geo.n_rot, dtype=torch.float64, device=dev)
    Wp_tot = torch.zeros(geo.n_rot * ps, dtype=torch.float64, device=dev)
    for ci, (g, Kc, off) in enumerate(chunks):
        nc, ds = g.n_data, g.data_stride
        G = torch.full((max(1, g.n_rot * ds),), float("nan"), dtype=torch.float32, device=dev)
        b = torch.empty(max(1, nc), dtype=torch.float64, device=dev)
        stats = torch.empty(max(1, 2 * nc), dtype=torch.float64, device=dev)
        P = torch.empty(max(1, g.n_rot * ds), dtype=g.p_dtype, device=dev)
        L = torch.empty(max(1, nc), dtype=torch.float64, device=dev)
        rho = torch.empty(geo.n_rot, dtype=torch.float64, device=dev)
        emc.emc_loglik(g, Kc, slices, scale, c, G, b)
        Gc = G.clone()
        emc.emc_responsibilities(g, G, S, b, emc.EMC_RESP_FULL, stats, P, L, rho)
        emc.emc_compress(g, P, Kc, rho, Wp, num, den, accumulate=ci > 0, ws=cws)
        if nc:
            rho_tot += rho
            Wp_tot += Wp.double()
            Gs.append(Gc[:g.n_rot * ds].view(g.n_rot, ds)[:, :nc].double())
            Ps.append(P[:g.n_rot * ds].view(g.n_rot, ds).double())
            bs.append(b[:nc])
            Ls.append(L[:nc])
            sts.append(stats[:2 * nc].view(nc, 2))
        # after compress the slice buffer holds W' when Wp aliases it; here it does not
    model_out = torch.empty(N3, dtype=torch.float32, device=dev)
    loglik = torch.empty(1, dtype=torch.float64, device=dev)
    L_all = torch.cat(Ls) if Ls else torch.empty(1, dtype=torch.float64, device=dev)
    emc.emc_finalize(geo, num, den, m, model_out, L_all, n, loglik)
    torch.cuda.synchronize()
    r = {k: v.detach().double().cpu().numpy() for k, v in out.items()}
    res = dict(c=r["c"][:geo.n_pix], S=r["S"], scale=r["scale"], num=num.cpu().numpy(), den=den.cpu().numpy(),
               model=model_out.double().cpu().numpy(), loglik=float(loglik.item()), rho=rho_tot.cpu().numpy())
    res["logW_c"] = r["A"][:, :geo.n_pix]
    res["logW_pad"] = r["A"][:, geo.n_pix:]
    res["Wp"] = Wp_tot.view(geo.n_rot, ps)[:, :geo.n_pix].cpu().numpy()
    if Gs:
        S_ = S.double()
        res["Q"] = torch.cat([G_ + b_[None, :] - S_[:, None] for G_, b_ in zip(Gs, bs)], dim=1).cpu().numpy()
        Pfull = [P_[:, :g.n_data] for P_, (g, _, _) in zip(Ps, [ch for ch in chunks if ch[0].n_data])]
        Ppad = [P_[:, g.n_data:] for P_, (g, _, _) in zip(Ps, [ch for ch in chunks if ch[0].n_data])]
        res["P"] = torch.cat(Pfull, dim=1).cpu().numpy()
        res["P_pad_max"] = max(float(x.abs().max()) if x.numel() else 0.0 for x in Ppad)
        res["L"] = torch.cat(Ls).cpu().numpy()
        res["stats"] = torch.cat(sts).cpu().numpy()
    return res


def q_rel_err(Q_gpu, Q_ref):
    """Worst frame of max_j |dQ_jk| / max_j |Q_jk|."""
    return float(np.max(np.max(np.abs(Q_gpu - Q_ref), axis=0) / np.max(np.abs(Q_ref), axis=0)))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def top1_agreement(P_gpu, P_ref, rel_tie=1e-3):
    """Fraction of frames whose most probable rotation agrees.

    Where the reference's best rotations are tied within `rel_tie` (relative)
    several answers are correct: a frame agrees when the GPU's choice has a
    reference probability within that margin of the reference maximum."""
    jg = np.argmax(P_gpu, axis=0)
    k = np.arange(P_ref.shape[1])
    return float(np.mean(P_ref[jg, k] >= (1.0 - rel_tie) * P_ref.max(axis=0)))


def top1_same_precision(P_gpu_bf16, P_ref):
    """Top-1 agreement with the decision taken in the kernel's precision on both
    sides: the reference responsibilities are rounded to BF16 (as the GPU stores
    them) before the arg-max; equal values go to the lower rotation index."""
    ref = torch.as_tensor(np.asarray(P_ref, np.float32)).to(torch.bfloat16).double().numpy()
    return float(np.mean(np.argmax(P_gpu_bf16, axis=0) == np.argmax(ref, axis=0)))


def top1_strict(P_gpu, P_ref):
    return float(np.mean(np.argmax(P_gpu, axis=0) == np.argmax(P_ref, axis=0)))


def candidate_pairs(buf, plan, n_rot, frames=None):
    """Every candidate (rotation, frame) pair of a proposal plan, with the element
    offsets of its log-likelihood sum in the G array and of its responsibility in
    the blocked P array (layouts of emc_proposed_workspace_view); only frames in
    `frames` when given.  Returns int64 numpy arrays (j, frame, g_off, p_off)."""
    pa = lambda addr, n, dt: emc.plan_array(buf, addr, n, dt).cpu().numpy()
    groups = pa(plan.groups, 4 * plan.n_groups, torch.int32).reshape(-1, 4).astype(np.int64)
    grp_off = pa(plan.grp_off, plan.n_groups + 1, torch.int64)
    cf_ptr = pa(plan.cf_ptr, plan.n_cells + 1, torch.int64)
    cf_frame = pa(plan.cf_frame, int(cf_ptr[-1]), torch.int32).astype(np.int64)
    cf_mask = pa(plan.cf_mask, int(cf_ptr[-1]), torch.int32).astype(np.int64) & 0xffffffff
    cand_frames = pa(plan.cand_frames, plan.n_cand, torch.int32).astype(np.int64)
    pack_rot = pa(plan.pack_rot, n_rot, torch.int32).astype(np.int64)
    rot_local = pa(plan.rot_local, n_rot, torch.int32).astype(np.int64)
    keep = None if frames is None else set(int(f) for f in frames)
    js, ks, go, po = [], [], [], []
    for g in range(plan.n_groups):
        c, first, cnt = groups[g, 0], groups[g, 1], groups[g, 2]
        fr = cand_frames[cf_frame[cf_ptr[c]:cf_ptr[c + 1]]]
        msk = cf_mask[cf_ptr[c]:cf_ptr[c + 1]]
        f = np.arange(fr.size)
        if keep is not None:
            sel = np.fromiter((int(x) in keep for x in fr), bool, fr.size)
            f, fr, msk = f[sel], fr[sel], msk[sel]
        if f.size == 0:
            continue
        r = np.arange(cnt)
        F, R = np.meshgrid(f, r, indexing="ij")
        # a pack's list holds the union of its cells' lists: only the pairs whose cell
        # the frame proposes are candidates
        cand = ((msk[:, None] >> rot_local[first + R]) & 1).astype(bool)
        F, R = F[cand], R[cand]
        js.append(pack_rot[first + R])
        ks.append(np.broadcast_to(fr[:, None], cand.shape)[cand])
        go.append(grp_off[g] + 32 * F + R)
        po.append(grp_off[g] + (F >> 5) * 1024 + R * 32 + (F & 31))
    cat = lambda a: np.concatenate(a) if a else np.zeros(0, np.int64)
    return cat(js), cat(ks), cat(go), cat(po)


def proposed_pairs_values(prop_ws, view, pairs):
    """(G, P) of the given pairs read from the workspace of the last proposed step."""
    _, _, go, po = pairs
    G = prop_ws[view.G:].view(torch.float32)
    P = prop_ws[view.P:view.P + 2 * (int(po.max()) + 1 if po.size else 1)].view(torch.bfloat16)
    gi = torch.as_tensor(go, device=prop_ws.device)
    pi = torch.as_tensor(po, device=prop_ws.device)
    return G[gi].double().cpu().numpy(), P[pi].double().cpu().numpy()
