"""Proposal network on the GPU vs its FP64 oracle: preprocessing, forward,
gradients, Adam, top-K and cell targets (FP32 kernels: relative error <= 1e-4)."""
import numpy as np
import pytest

from oracle import cnn_oracle as C

pytestmark = pytest.mark.gpu

N_CELLS = 37


def _flat(p, n_cells):
    parts = []
    for l in range(4):
        parts += [p[f"w{l}"].ravel(), p[f"b{l}"].ravel()]
    parts += [p["wf"].ravel(), p["bf"].ravel()]
    return np.concatenate(parts)


def _unflat(v, n_cells):
    p, o = {}, 0
    for l in range(4):
        ci, co = C.CHANNELS[l], C.CHANNELS[l + 1]
        p[f"w{l}"] = v[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        p[f"b{l}"] = v[o:o + co]
        o += co
    p["wf"] = v[o:o + n_cells * 2048].reshape(n_cells, 2048)
    o += n_cells * 2048
    p["bf"] = v[o:o + n_cells]
    return p


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-30))


@pytest.fixture(scope="module")
def setup(gpu_lib):
    import torch

    emc = gpu_lib
    rng = np.random.default_rng(11)
    p = C.init_params(rng, N_CELLS)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.05
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    assert _flat(p, N_CELLS).size == emc.emc_cnn_param_count(N_CELLS)
    B = 6
    x = np.log1p(rng.poisson(1.0, size=(B, 1, 64, 64))).astype(np.float32).astype(np.float64)
    T = rng.dirichlet(np.ones(N_CELLS) * 0.3, size=B).astype(np.float32).astype(np.float64)
    dev = dict(p=torch.as_tensor(_flat(p, N_CELLS), dtype=torch.float32, device="cuda"),
               x=torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous(),
               T=torch.as_tensor(T, dtype=torch.float32, device="cuda").contiguous(),
               ws=torch.empty(emc.emc_cnn_workspace_bytes(N_CELLS, B), dtype=torch.uint8, device="cuda"))
    return emc, p, x, T, B, dev


def test_cnn_forward_matches_oracle(setup):
    import torch

    emc, p, x, T, B, d = setup
    z = torch.empty(B * N_CELLS, dtype=torch.float32, device="cuda")
    emc.emc_cnn_forward(N_CELLS, d["p"], d["x"], B, z, d["ws"])
    zr, _ = C.forward(p, x)
    assert _rel(z.double().cpu().numpy().reshape(B, N_CELLS), zr) <= 1e-4


def test_cnn_gradients_match_oracle(setup):
    import torch

    emc, p, x, T, B, d = setup
    g = torch.empty_like(d["p"])
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    emc.emc_cnn_gradients(N_CELLS, d["p"], d["x"], d["T"], B, g, loss, d["ws"])
    z, acts = C.forward(p, x)
    gr = C.backward(p, acts, z, T)
    assert abs(loss.item() - C.loss(z, T)) <= 1e-5 * abs(C.loss(z, T))
    gg = _unflat(g.double().cpu().numpy(), N_CELLS)
    for k in gr:
        assert _rel(gg[k], gr[k]) <= 1e-4, (k, _rel(gg[k], gr[k]))


@pytest.mark.parametrize("B", [1, 40, 70])
def test_cnn_gradients_match_oracle_larger_batches(gpu_lib, B):
    """Batches that split every weight-gradient reduction over several ranges and
    leave ragged output tiles in the contractions, against the FP64 oracle's
    gradients."""
    import torch

    emc = gpu_lib
    n_cells = 150
    rng = np.random.default_rng(21 + B)
    p = C.init_params(rng, n_cells)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.05
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    x = np.log1p(rng.poisson(1.0, size=(B, 1, 64, 64))).astype(np.float32).astype(np.float64)
    T = rng.dirichlet(np.ones(n_cells) * 0.3, size=B).astype(np.float32).astype(np.float64)
    dp = torch.as_tensor(_flat(p, n_cells), dtype=torch.float32, device="cuda")
    ws = torch.empty(emc.emc_cnn_workspace_bytes(n_cells, B), dtype=torch.uint8, device="cuda")
    g = torch.empty_like(dp)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    emc.emc_cnn_gradients(n_cells, dp, torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous(),
                          torch.as_tensor(T, dtype=torch.float32, device="cuda").contiguous(), B, g, loss, ws)
    z, acts = C.forward(p, x)
    gr = C.backward(p, acts, z, T)
    gg = _unflat(g.double().cpu().numpy(), n_cells)
    errs = {k: _rel(gg[k], gr[k]) for k in gr}
    print(f"\n[cnn B={B}] loss {loss.item():.6f} (oracle {C.loss(z, T):.6f}); gradient rel errors "
          + " ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    assert abs(loss.item() - C.loss(z, T)) <= 1e-5 * abs(C.loss(z, T))
    for k, e in errs.items():
        assert e <= 1e-4, (k, e)


def test_cnn_adam_matches_oracle(setup):
    import torch

    emc, p, x, T, B, d = setup
    rng = np.random.default_rng(12)
    n = emc.emc_cnn_param_count(N_CELLS)
    params = d["p"].clone()
    m = torch.zeros(n, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    pr = {k: a.copy() for k, a in p.items()}
    state = {}
    for step in (1, 2, 3):
        gv = rng.standard_normal(n).astype(np.float32).astype(np.float64)
        emc.emc_cnn_adam(N_CELLS, params, torch.as_tensor(gv, dtype=torch.float32, device="cuda"), m, v, step, 1e-3)
        C.adam_step(pr, _unflat(gv, N_CELLS), state, lr=1e-3)
    torch.cuda.synchronize()
    got = params.double().cpu().numpy()
    ref = _flat(pr, N_CELLS)
    base = _flat(p, N_CELLS)
    assert np.max(np.abs((got - base) - (ref - base))) <= 1e-6


def test_cnn_training_steps_reduce_loss(setup):
    import torch

    emc, p, x, T, B, d = setup
    n = emc.emc_cnn_param_count(N_CELLS)
    params = d["p"].clone()
    g = torch.empty_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    losses = []
    for step in range(1, 31):
        emc.emc_cnn_gradients(N_CELLS, params, d["x"], d["T"], B, g, loss, d["ws"])
        losses.append(loss.item())
        emc.emc_cnn_adam(N_CELLS, params, g, m, v, step, 1e-3)
    assert losses[-1] < 0.8 * losses[0], losses


def test_topk_matches_stable_argsort(gpu_lib):
    import torch

    emc = gpu_lib
    rng = np.random.default_rng(13)
    z = rng.standard_normal((50, 2000)).astype(np.float32)
    z[3, 100:110] = 5.0                      # ties: lower index first
    out = torch.empty(50 * 64, dtype=torch.int32, device="cuda")
    emc.emc_cnn_topk(torch.as_tensor(z, device="cuda"), 50, 2000, 64, out)
    np.testing.assert_array_equal(out.cpu().numpy().reshape(50, 64), C.topk_cells(z.astype(np.float64), 64))


def test_preprocess_and_targets_match_oracle(gpu_lib):
    import torch

    from emc_inputs import WORKLOADS, detector_mask, detector_q, proposal_bins, scaled
    from gpu_helpers import geometry, pack, upload_counts

    emc = gpu_lib
    wl = scaled(WORKLOADS[2], n_rot=300, n_data=70)
    q, _ = detector_q(wl)
    mask = detector_mask(wl)
    rng = np.random.default_rng(14)
    counts = (rng.poisson(0.3, size=(70, wl.n_pix)) * mask[None, :]).astype(np.uint16)
    quat = rng.standard_normal((300, 4))
    log_w = np.full(300, -np.log(300))
    bins = proposal_bins(wl.det_n, mask)
    for prec in (0, 1):
        geo = geometry(wl.grid_n, q, mask, quat, log_w, 70, prec)
        K = pack(geo, upload_counts(counts))
        x = torch.empty(70 * 4096, dtype=torch.float32, device="cuda")
        emc.emc_cnn_preprocess(geo, K, torch.as_tensor(bins, device="cuda"), None, 70, x)
        np.testing.assert_allclose(x.double().cpu().numpy().reshape(70, 1, 64, 64), C.bin_log(counts, bins),
                                   rtol=1e-6, atol=1e-6)
        # targets from random responsibilities
        cell_of = rng.integers(0, 20, size=300)
        order = np.argsort(cell_of, kind="stable")
        ptr = np.concatenate([[0], np.cumsum(np.bincount(cell_of, minlength=20))]).astype(np.int32)
        P = rng.dirichlet(np.ones(300), size=70).T                                  # [j][k]
        Pd = torch.zeros(300 * geo.data_stride, dtype=geo.p_dtype, device="cuda")
        Pd.view(300, -1)[:, :70] = torch.as_tensor(P, dtype=geo.p_dtype)
        Pq = Pd.view(300, -1)[:, :70].double().cpu().numpy()
        T = torch.empty(70 * 20, dtype=torch.float32, device="cuda")
        emc.emc_cell_targets(geo, Pd, torch.as_tensor(ptr, device="cuda"),
                             torch.as_tensor(order.astype(np.int32), device="cuda"), 20, T)
        np.testing.assert_allclose(T.double().cpu().numpy().reshape(70, 20), C.cell_targets(Pq, cell_of, 20),
                                   rtol=1e-5, atol=1e-7)
