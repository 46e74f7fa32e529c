"""Helpers for the GPU parity tests: run the C-ABI entry points on device tensors
and bring every intermediate back as float64 numpy arrays in the oracle's index
order.  Comparison metrics follow the tolerances of the plain FP32 path."""
from __future__ import annotations

import numpy as np
import torch

from paper_1409_4256_amd import emc


def geometry(grid_n, q, mask, quat, log_w, n_data):
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dt)
    return emc.Geometry(grid_n, t(q, torch.float64), t(mask, torch.uint8), t(quat, torch.float64),
                        t(log_w, torch.float64), n_data)


def upload_counts(counts):
    if isinstance(counts, torch.Tensor):
        return counts.to("cuda").contiguous()
    return torch.from_numpy(np.ascontiguousarray(counts.astype(np.uint16))).to("cuda")


def pack(geo, counts_dev):
    K = torch.empty(max(1, geo.n_data * geo.pix_stride), dtype=torch.float32, device="cuda")
    emc.emc_pack_frames(geo, counts_dev, K)
    return K


def run_steps(geo, model, K, frame_chunk=None):
    """expand -> loglik -> responsibilities -> compress (optionally in frame chunks) -> finalize."""
    dev = "cuda"
    N3 = geo.grid_n ** 3
    ps, rs = geo.pix_stride, geo.rot_stride
    n = geo.n_data
    m = torch.as_tensor(np.asarray(model, dtype=np.float32)).to(dev)
    c = torch.empty(ps, dtype=torch.float64, device=dev)
    logW = torch.empty(geo.n_rot * ps, dtype=torch.float32, device=dev)
    S = torch.empty(geo.n_rot, dtype=torch.float64, device=dev)
    emc.emc_expand(geo, m, c, logW, S)
    out = dict(c=c, logW=logW.clone(), S=S)
    G = torch.full((max(1, n * rs),), float("nan"), dtype=torch.float32, device=dev)
    b = torch.empty(max(1, n), dtype=torch.float64, device=dev)
    stats = torch.empty(max(1, 2 * n), dtype=torch.float64, device=dev)
    P = torch.empty_like(G)
    L = torch.empty(max(1, n), dtype=torch.float64, device=dev)
    num = torch.empty(N3, dtype=torch.float64, device=dev)
    den = torch.empty(N3, dtype=torch.float64, device=dev)
    Wp = torch.empty(geo.n_rot * ps, dtype=torch.float32, device=dev)
    rho_tot = torch.zeros(geo.n_rot, dtype=torch.float64, device=dev)
    chunk = n if not frame_chunk else frame_chunk
    starts = list(range(0, n, chunk)) if n else [0]
    Wp_tot = torch.zeros(geo.n_rot * ps, dtype=torch.float64, device=dev)
    for ci, s in enumerate(starts):
        nc = min(chunk, n - s) if n else 0
        g = geo.with_frames(nc)
        Kc = K[s * ps:(s + nc) * ps] if nc else K
        Gc = G[s * rs:(s + nc) * rs] if nc else G
        Pc = P[s * rs:(s + nc) * rs] if nc else P
        rho = torch.empty(geo.n_rot, dtype=torch.float64, device=dev)
        emc.emc_loglik(g, Kc, logW, c, Gc, b[s:s + nc] if nc else b)
        emc.emc_responsibilities(g, Gc, S, b[s:s + nc] if nc else b, emc.EMC_RESP_FULL,
                                 stats[2 * s:2 * (s + nc)] if nc else stats, Pc, L[s:s + nc] if nc else L, rho)
        emc.emc_compress(g, Pc, Kc, rho, Wp, num, den, accumulate=ci > 0)
        rho_tot += rho
        Wp_tot += Wp.double() if nc else 0
    model_out = torch.empty(N3, dtype=torch.float32, device=dev)
    loglik = torch.empty(1, dtype=torch.float64, device=dev)
    emc.emc_finalize(geo, num, den, m, model_out, L, n, loglik)
    torch.cuda.synchronize()
    out.update(G=G, b=b, stats=stats, P=P, L=L, rho=rho_tot, Wp=Wp_tot, num=num, den=den, model=model_out,
               loglik=loglik)
    return to_oracle_order(geo, out)


def to_oracle_order(geo, out):
    n, nr, npx, ps, rs = geo.n_data, geo.n_rot, geo.n_pix, geo.pix_stride, geo.rot_stride
    h = {k: v.detach().double().cpu().numpy() for k, v in out.items()}
    r = dict(c=h["c"][:npx], S=h["S"], num=h["num"], den=h["den"], model=h["model"],
             loglik=float(h["loglik"][0]), rho=h["rho"])
    r["logW_c"] = h["logW"].reshape(nr, ps)[:, :npx]                      # log W - c
    r["logW_pad"] = h["logW"].reshape(nr, ps)[:, npx:]
    r["Wp"] = h["Wp"].reshape(nr, ps)[:, :npx]
    if n:
        G = h["G"][:n * rs].reshape(n, rs)[:, :nr]
        r["Q"] = (G + h["b"][:n, None] - h["S"][None, :]).T             # [j][k]
        r["P"] = h["P"][:n * rs].reshape(n, rs)[:, :nr].T               # [j][k]
        r["P_pad"] = h["P"][:n * rs].reshape(n, rs)[:, nr:]
        r["L"] = h["L"][:n]
        r["stats"] = h["stats"][:2 * n].reshape(n, 2)
    return r


def q_rel_err(Q_gpu, Q_ref):
    """Worst frame of max_j |dQ_jk| / max_j |Q_jk|."""
    return float(np.max(np.max(np.abs(Q_gpu - Q_ref), axis=0) / np.max(np.abs(Q_ref), axis=0)))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
