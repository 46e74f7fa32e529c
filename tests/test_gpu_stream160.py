"""Frame-chunk streaming at the largest share: 160^3 grid, 128x128 detector,
100000 rotations, 500000 frames at ~1000 photons in ten 50000-frame chunks,
BF16 form (each chunk's E-step is independent; the numerator and denominator
grids accumulate over chunks before the one division, the k-direction split of
Section 3.3).

Checked against the FP64 oracle one by one where it can compute (slices of
sampled rotations; log-likelihoods of sampled (rotation, frame) pairs from the
first and the last chunk) and by identities that hold at any size."""
import numpy as np
import pytest

import oracle as O
from emc_inputs import WORKLOADS, make_inputs

pytestmark = pytest.mark.gpu

CHUNK = 50000


@pytest.fixture(scope="module")
def streamed(gpu_lib):
    import torch

    emc = gpu_lib
    wl = WORKLOADS[5]
    print("\n[stream160] generating 160^3 / 100000 rotations / 500000 frames on the GPU", flush=True)
    inp = make_inputs(wl, device="cuda", with_truth=False)
    dev = "cuda"
    geo = emc.Geometry(wl.grid_n, torch.as_tensor(inp.q), torch.as_tensor(inp.mask), torch.as_tensor(inp.quat),
                       torch.as_tensor(inp.log_w), wl.n_data, emc.EMC_PREC_BF16)
    ps = geo.pix_stride
    N3 = wl.grid_n ** 3
    model = torch.as_tensor(inp.model_start, dtype=torch.float32, device=dev)
    c = torch.empty(ps, dtype=torch.float64, device=dev)
    slices = emc.slices_tensor(geo)
    S = torch.empty(wl.n_rot, dtype=torch.float64, device=dev)
    scale = torch.empty(wl.n_rot, dtype=torch.float32, device=dev)
    emc.emc_expand(geo, model, c, slices, S, scale)
    rng = np.random.default_rng(5)
    js = np.sort(rng.choice(wl.n_rot, 24, replace=False))
    jt = torch.as_tensor(js, device=dev)
    hl = slices.view(torch.bfloat16)
    A = ((hl[:wl.n_rot * ps].view(wl.n_rot, ps)[jt].double() + hl[wl.n_rot * ps:2 * wl.n_rot * ps].view(
        wl.n_rot, ps)[jt].double()) * scale[jt].double()[:, None]).cpu().numpy()
    gc = geo.with_frames(CHUNK)
    ds = gc.data_stride
    G = torch.empty(wl.n_rot * ds, dtype=torch.float32, device=dev)
    P = torch.empty(wl.n_rot * ds, dtype=torch.bfloat16, device=dev)
    b = torch.empty(CHUNK, dtype=torch.float64, device=dev)
    stats = torch.empty(2 * CHUNK, dtype=torch.float64, device=dev)
    L = torch.empty(wl.n_data, dtype=torch.float64, device=dev)
    rho = torch.empty(wl.n_rot, dtype=torch.float64, device=dev)
    rho_tot = torch.zeros(wl.n_rot, dtype=torch.float64, device=dev)
    Wp = torch.empty(wl.n_rot * ps, dtype=torch.float32, device=dev)
    num = torch.empty(N3, dtype=torch.float64, device=dev)
    den = torch.empty(N3, dtype=torch.float64, device=dev)
    K = emc.frames_tensor(gc)
    frames = torch.arange(wl.n_data, dtype=torch.int32, device=dev)
    out = dict(js=js, A=A, c=c.cpu().numpy(), S=S.cpu().numpy(), G={}, b={}, ks={}, Kr={}, colsum=[])
    n_chunks = wl.n_data // CHUNK
    cws = torch.empty(emc.emc_compress_workspace_bytes(geo), dtype=torch.uint8, device="cuda")
    for ci in range(n_chunks):
        emc.emc_pack_frames_list(gc, inp.counts, frames[ci * CHUNK:(ci + 1) * CHUNK], K)
        emc.emc_loglik(gc, K, slices, scale, c, G, b)
        if ci in (0, n_chunks - 1):
            ks = np.sort(rng.choice(CHUNK, 12, replace=False))
            kt = torch.as_tensor(ks, device=dev)
            torch.cuda.synchronize()
            out["G"][ci] = G.view(wl.n_rot, ds)[jt][:, kt].double().cpu().numpy()
            out["b"][ci] = b[kt].cpu().numpy()
            out["ks"][ci] = ks
            out["Kr"][ci] = inp.counts.view(torch.int16)[kt + ci * CHUNK].to(torch.int32).cpu().numpy()
        emc.emc_responsibilities(gc, G, S, b, emc.EMC_RESP_FULL, stats, P, L[ci * CHUNK:(ci + 1) * CHUNK], rho)
        out["colsum"].append(P.view(wl.n_rot, ds)[:, :CHUNK].double().sum(0).cpu().numpy())
        emc.emc_compress(gc, P, K, rho, Wp, num, den, accumulate=ci > 0, ws=cws)
        rho_tot += rho
        print(f"[stream160] chunk {ci + 1}/{n_chunks} done", flush=True)
    m_out = torch.empty_like(model)
    loglik = torch.empty(1, dtype=torch.float64, device=dev)
    emc.emc_finalize(geo, num, den, model, m_out, L, wl.n_data, loglik)
    torch.cuda.synchronize()
    out.update(num_sum=float(num.sum().item()), den_sum=float(den.sum().item()), rho_sum=float(rho_tot.sum().item()),
               photons=float(inp.counts.to(torch.int64).sum().item()), loglik=loglik.item(),
               model_in=model.double().cpu().numpy(), model_out=m_out.double().cpu().numpy(),
               den_pos=(den > 0).cpu().numpy())
    return inp, out


def test_stream160_slices_and_loglik_pairs(streamed):
    inp, s = streamed
    wl = inp.wl
    v = np.flatnonzero(inp.mask)
    q = np.asarray(inp.q, np.float32).astype(np.float64)
    quat = np.asarray(inp.quat, np.float32).astype(np.float64)[s["js"]]
    W = O.expand(s["model_in"], q[v], quat, wl.grid_n)
    assert np.max(np.abs(s["A"][:, v] + s["c"][None, v] - np.log(np.maximum(W, 1e-10)))) < 2e-4
    np.testing.assert_allclose(s["S"][s["js"]], np.maximum(W, 1e-10).sum(1), rtol=1e-12)
    Wfull = np.zeros((W.shape[0], wl.n_pix))
    Wfull[:, v] = W
    for ci in s["G"]:
        Q_ref = O.log_likelihood(Wfull, s["Kr"][ci], inp.mask)
        Q_gpu = s["G"][ci] + s["b"][ci][None, :] - s["S"][s["js"]][:, None]
        rel = np.max(np.abs(Q_gpu - Q_ref), axis=0) / np.max(np.abs(Q_ref), axis=0)
        print(f"\n[stream160] chunk {ci}: log-likelihood relative error {rel.max():.2e}")
        assert rel.max() <= 2e-4


def test_stream160_identities(streamed):
    inp, s = streamed
    wl = inp.wl
    nv = int(np.asarray(inp.mask).sum())
    for cs in s["colsum"]:
        np.testing.assert_allclose(cs, 1.0, atol=2e-2)
    np.testing.assert_allclose(s["rho_sum"], wl.n_data, rtol=1e-3)
    np.testing.assert_allclose(s["den_sum"], s["rho_sum"] * nv, rtol=1e-9)
    np.testing.assert_allclose(s["num_sum"], s["photons"], rtol=1e-3)
    m = s["model_out"]
    assert np.all(np.isfinite(m)) and np.all(m[s["den_pos"]] >= 0)
    np.testing.assert_array_equal(m[~s["den_pos"]], s["model_in"][~s["den_pos"]])
    assert np.isfinite(s["loglik"])
