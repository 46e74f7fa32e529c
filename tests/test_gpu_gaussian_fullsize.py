"""Gaussian-model iteration at the full one-GPU share (128^3 grid, 16384 pixels,
25000 rotations, 100000 frames), with the benchmark's geometry, packed frames and
brick-major c-step.

The FP64 oracle computes what it can pair by pair: the slices of sampled
rotations, hence the fluence update (eq. (2.6)) and the log-likelihood (eq. (2.3))
of sampled (rotation, frame) pairs.  The responsibilities are held to what holds
at any size: each frame's sum to one, and log P_jk - log P_j'k equals
a_jk - a_j'k (eq. (2.4)), which needs no normalisation."""
import numpy as np
import pytest

from emc_inputs import WORKLOADS, make_inputs
from oracle import emc_oracle as O
from oracle import gauss_oracle as GO

pytestmark = pytest.mark.gpu


def test_gaussian_full_share(gpu_lib):
    import torch

    import bench

    emc = gpu_lib
    print("\n[gaussian fullsize] generating 128^3 / 25000 rotations / 100000 frames on the GPU", flush=True)
    inp = make_inputs(WORKLOADS[2], device="cuda", with_truth=False)
    run = bench.Run(inp, emc.EMC_PREC_FP32)
    g, wl = run.geo, inp.wl
    n, ds, N = wl.n_data, g.data_stride, wl.grid_n
    sigma = 2.0
    phi = torch.empty(wl.n_rot * ds, dtype=torch.float32, device="cuda")
    P = torch.empty(wl.n_rot * ds, dtype=torch.float32, device="cuda")
    ws = torch.empty(emc.emc_gaussian_workspace_bytes(g), dtype=torch.uint8, device="cuda")
    m_out = torch.empty_like(run.model[0])
    ll = torch.empty(1, dtype=torch.float64, device="cuda")
    print("[gaussian fullsize] iteration", flush=True)
    emc.emc_iterate_gaussian(g, sigma, run.model[0], run.K, phi, True, m_out, ll, P_out=P, ws=ws)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    ks = np.sort(rng.choice(n, 12, replace=False))
    kt = torch.as_tensor(ks, device="cuda")
    Pv = P.view(wl.n_rot, ds)
    colsum = Pv[:, :n].double().sum(0).cpu().numpy()
    np.testing.assert_allclose(colsum, 1.0, atol=1e-4)
    Pk = Pv[:, kt].double().cpu().numpy()                                   # [n_rot][12]
    phik = phi.view(wl.n_rot, ds)[:, kt].double().cpu().numpy()
    js = np.unique(np.concatenate([rng.choice(wl.n_rot, 24, replace=False), Pk.argmax(axis=0)]))
    print(f"[gaussian fullsize] oracle slices of {len(js)} rotations", flush=True)
    q = np.asarray(inp.q, np.float32).astype(np.float64)
    quat = np.asarray(inp.quat, np.float32).astype(np.float64)
    model = run.model[0].double().cpu().numpy()
    W = O.expand(model, q, quat[js], N)                                      # [len(js)][n_pix]
    if isinstance(inp.counts, torch.Tensor):      # row views (no device indexing of uint16)
        counts = np.stack([inp.counts[int(k)].cpu().numpy() for k in ks])
    else:
        counts = inp.counts[ks]
    mask = np.asarray(inp.mask.cpu() if isinstance(inp.mask, torch.Tensor) else inp.mask)
    phi_o = GO.fluence(W, counts, mask)                                     # [len(js)][12]
    err_phi = np.max(np.abs(phik[js] - phi_o) / phi_o)
    Q = GO.log_likelihood(W, counts, mask, phi_o, sigma)                    # first iteration: own fluence
    a = Q + np.asarray(inp.log_w)[js][:, None]
    # log-ratio of responsibilities against the frame's most probable sampled rotation,
    # where both are representable in FP32 (within e^-60 of it)
    lp = np.log(np.maximum(Pk[js], 1e-300))
    ref = np.argmax(a, axis=0)
    d_gpu = lp - lp[ref, np.arange(len(ks))]
    d_or = a - a[ref, np.arange(len(ks))]
    use = d_or > -60.0
    err_a = np.max(np.abs(d_gpu[use] - d_or[use]))
    print(f"[gaussian fullsize] phi max rel {err_phi:.2e}, log P ratio max abs {err_a:.2e} over {use.sum()} pairs, "
          f"loglik {ll.item():.4f}", flush=True)
    assert err_phi <= 1e-5
    assert err_a <= 2e-3                      # log of FP32-stored P (relative 6e-8) and FP32 contraction
    np.testing.assert_array_equal(np.argmax(Pk[js], axis=0), ref)
    assert np.isfinite(ll.item())
    assert torch.isfinite(m_out).all().item()
